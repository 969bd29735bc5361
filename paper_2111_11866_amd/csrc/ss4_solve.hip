// Time-step kernels: assembly of the finite-volume system from
// reduced-diamond-cell face gradients (Sec. 3.2.2, the uniform-h system with
// A_eps and A_eps-bar), red-black SOR half-sweeps with the residual norm fused
// in, and the host driver of the iteration.
#include <cmath>

#include "ss4_internal.hpp"

namespace ss4 {
namespace {

constexpr int kSplit = 0;    // assembly output for the solver (colour-split)
constexpr int kNatural = 1;  // assembly output in the natural layout (export)

struct AsmArgs {
    Layout L;
    double th2;       // tau / h^2
    double eps2;      // eps^2
    double inv_h;
    const double* G;  // 4 x padded
    const double* w;  // padded u^{resc;n-1}
    double* ured0;
    double* ured1;
    double* ublack;
    double* coef;     // 16 arrays of csplit: [colour*8 + face]
    double* rhs;      // 2 arrays of csplit
    double* coef_nat; // interior x 8
    double* b_nat;    // interior
    double* part_a;
    double* part_b;
    Ctrl* C;
};

// One thread per padded cell.  Ghost cells only copy their Dirichlet value
// into the colour-split u; interior cells compute the 8 coefficients from the
// 33-point neighbourhood of w and G on the 8 faces.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_assemble(AsmArgs a)
{
    __shared__ double lds[4];
    __shared__ int flag;
    const Layout& L = a.L;
    const int64_t s1 = 1, s2 = L.p1, s3 = (int64_t)L.p1 * L.p2, s4 = s3 * L.p3;
    const int64_t sd[4] = {s1, s2, s3, s4};
    double acc_b = 0.0, acc_r = 0.0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < L.npad; p += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(p % L.p1);
        const int64_t prow = p / L.p1;
        const int j = (int)(prow % L.p2);
        const int64_t t2 = prow / L.p2;
        const int k = (int)(t2 % L.p3);
        const int l = (int)(t2 / L.p3);
        const int colour = (i + j + k + l) & 1;
        const int m = (i - 1) >> 1;
        const double w0 = a.w[p];
        if (MODE == kSplit) {
            const int64_t us = prow * L.rs + L.xoff + m;
            if (colour == 0) { a.ured0[us] = w0; a.ured1[us] = w0; }
            else a.ublack[us] = w0;
        }
        const bool inside = i >= 1 && i <= L.n1 && j >= 1 && j <= L.n2 && k >= 1 && k <= L.n3 && l >= 1 && l <= L.n4;
        if (!inside) continue;
        const int idx[4] = {i, j, k, l};
        const int nn[4] = {L.n1, L.n2, L.n3, L.n4};
        // face neighbours
        double wm[4], wp[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) { wm[d] = a.w[p - sd[d]]; wp[d] = a.w[p + sd[d]]; }
        double q[8];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const double gnm = (w0 - wm[d]) * a.inv_h;   // normal, -e_d face
            const double gnp = (wp[d] - w0) * a.inv_h;   // normal, +e_d face
            double qm = gnm * gnm, qp = gnp * gnp;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t == d) continue;
                const double wpt = a.w[p + sd[t]], wmt = a.w[p - sd[t]];
                const double dm_pt = a.w[p - sd[d] + sd[t]], dm_mt = a.w[p - sd[d] - sd[t]];
                const double dp_pt = a.w[p + sd[d] + sd[t]], dp_mt = a.w[p + sd[d] - sd[t]];
                const double tm = ((dm_pt + wpt) - (dm_mt + wmt)) * (0.25 * a.inv_h);
                const double tp = ((wpt + dp_pt) - (wmt + dp_mt)) * (0.25 * a.inv_h);
                qm += tm * tm;
                qp += tp * tp;
            }
            q[2 * d] = qm;
            q[2 * d + 1] = qp;
        }
        double qs = 0.0;
#pragma unroll
        for (int f = 0; f < 8; ++f) qs += q[f];
        const double abar = sqrt(a.eps2 + qs / 8.0);
        const double scale = a.th2 * abar;
        double c[8];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const double gm = a.G[(int64_t)d * L.npad + p - sd[d]];
            const double gp = a.G[(int64_t)d * L.npad + p];
            c[2 * d] = scale * gm / sqrt(a.eps2 + q[2 * d]);
            c[2 * d + 1] = scale * gp / sqrt(a.eps2 + q[2 * d + 1]);
        }
        double D = 1.0;
#pragma unroll
        for (int f = 0; f < 8; ++f) D += c[f];
        double bfull = w0, off = 0.0;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            off += c[2 * d] * wm[d] + c[2 * d + 1] * wp[d];
            if (idx[d] == 1) bfull += c[2 * d] * wm[d];
            if (idx[d] == nn[d]) bfull += c[2 * d + 1] * wp[d];
        }
        const double r0 = (w0 + off) - D * w0;
        acc_b += bfull * bfull;
        acc_r += r0 * r0;
        const int64_t irow = ((int64_t)(l - 1) * L.n3 + (k - 1)) * L.n2 + (j - 1);
        if (MODE == kSplit) {
            const int64_t ci = irow * L.rsc + m;
#pragma unroll
            for (int f = 0; f < 8; ++f) a.coef[(int64_t)(colour * 8 + f) * L.csplit + ci] = c[f];
            a.rhs[(int64_t)colour * L.csplit + ci] = w0;
        } else {
            const int64_t qi = irow * L.n1 + (i - 1);
#pragma unroll
            for (int f = 0; f < 8; ++f) a.coef_nat[qi * 8 + f] = c[f];
            a.b_nat[qi] = bfull;
        }
    }
    if (MODE != kSplit) return;
    const double bb = block_sum(acc_b, lds);
    const double rr = block_sum(acc_r, lds);
    if (threadIdx.x == 0) { a.part_a[blockIdx.x] = bb; a.part_b[blockIdx.x] = rr; }
    if (!arrive_last(&a.C->arrive[0], gridDim.x, &flag)) return;
    const double B2 = sum_partials(a.part_a, gridDim.x, lds);
    const double R2 = sum_partials(a.part_b, gridDim.x, lds);
    if (threadIdx.x == 0) {
        Ctrl* C = a.C;
        C->bn = sqrt(B2);
        const double R = sqrt(R2);
        C->rel_res = C->bn > 0.0 ? R / C->bn : R;
        C->iterations = 0;
        C->final_red = 0;
        if (!(R2 < INFINITY) || !(B2 < INFINITY)) { C->status = SUBSURF4D_ENONFINITE; C->done = 1; }
        else if (R <= C->tol * C->bn) C->done = 1;
        else if (C->max_iter <= 0) { C->status = SUBSURF4D_NOT_CONVERGED; C->done = 1; }
        C->arrive[0] = 0;
    }
}

// Load an externally given system (natural layout, Dirichlet terms in b) into
// the colour-split arrays; ghost slots of u are 0 so they contribute nothing.
__global__ __launch_bounds__(kBlock) void k_load_system(Layout L, const double* coef_nat, const double* b_nat,
                                                         const double* u, double* ured0, double* ured1,
                                                         double* ublack, double* coef, double* rhs,
                                                         double* part_a, double* part_b, Ctrl* C)
{
    __shared__ double lds[4];
    __shared__ int flag;
    const int64_t sd[4] = {1, L.p1, (int64_t)L.p1 * L.p2, (int64_t)L.p1 * L.p2 * L.p3};
    double acc_b = 0.0, acc_r = 0.0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < L.npad; p += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(p % L.p1);
        const int64_t prow = p / L.p1;
        const int j = (int)(prow % L.p2);
        const int64_t t2 = prow / L.p2;
        const int k = (int)(t2 % L.p3);
        const int l = (int)(t2 / L.p3);
        const int colour = (i + j + k + l) & 1;
        const int m = (i - 1) >> 1;
        const bool inside = i >= 1 && i <= L.n1 && j >= 1 && j <= L.n2 && k >= 1 && k <= L.n3 && l >= 1 && l <= L.n4;
        const double v = inside ? u[p] : 0.0;
        const int64_t us = prow * L.rs + L.xoff + m;
        if (colour == 0) { ured0[us] = v; ured1[us] = v; }
        else ublack[us] = v;
        if (!inside) continue;
        const int idx[4] = {i, j, k, l};
        const int nn[4] = {L.n1, L.n2, L.n3, L.n4};
        const int64_t irow = ((int64_t)(l - 1) * L.n3 + (k - 1)) * L.n2 + (j - 1);
        const int64_t qi = irow * L.n1 + (i - 1);
        const int64_t ci = irow * L.rsc + m;
        double D = 1.0, s = b_nat[qi];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const double cm = coef_nat[qi * 8 + 2 * d], cp = coef_nat[qi * 8 + 2 * d + 1];
            coef[(int64_t)(colour * 8 + 2 * d) * L.csplit + ci] = cm;
            coef[(int64_t)(colour * 8 + 2 * d + 1) * L.csplit + ci] = cp;
            D += cm;
            D += cp;
            if (idx[d] > 1) s += cm * u[p - sd[d]];
            if (idx[d] < nn[d]) s += cp * u[p + sd[d]];
        }
        rhs[(int64_t)colour * L.csplit + ci] = b_nat[qi];
        const double r0 = s - D * v;
        acc_b += b_nat[qi] * b_nat[qi];
        acc_r += r0 * r0;
    }
    const double bb = block_sum(acc_b, lds);
    const double rr = block_sum(acc_r, lds);
    if (threadIdx.x == 0) { part_a[blockIdx.x] = bb; part_b[blockIdx.x] = rr; }
    if (!arrive_last(&C->arrive[0], gridDim.x, &flag)) return;
    const double B2 = sum_partials(part_a, gridDim.x, lds);
    const double R2 = sum_partials(part_b, gridDim.x, lds);
    if (threadIdx.x == 0) {
        C->bn = sqrt(B2);
        const double R = sqrt(R2);
        C->rel_res = C->bn > 0.0 ? R / C->bn : R;
        C->iterations = 0;
        C->final_red = 0;
        if (!(R2 < INFINITY) || !(B2 < INFINITY)) { C->status = SUBSURF4D_ENONFINITE; C->done = 1; }
        else if (R <= C->tol * C->bn) C->done = 1;
        else if (C->max_iter <= 0) { C->status = SUBSURF4D_NOT_CONVERGED; C->done = 1; }
        C->arrive[0] = 0;
    }
}

struct SweepArgs {
    Layout L;
    const double* uin;    // own colour, iterate k-1
    double* uout;         // own colour, iterate k (== uin for black)
    const double* uoth;   // other colour
    const double* coef;   // 8 arrays of csplit for this colour
    const double* rhs;    // this colour
    double omega;
    double* part;         // this kernel's per-block partials
    const double* part_other;  // black partials of iterate k-1 (red check)
    Ctrl* C;
    int k;                // iteration number
    int check;            // red: test the stopping rule for iterate k-1
};

// Half-sweep of colour COLOR (0 = red, 1 = black).  Tile = 64 slots of one row
// per wave, 4 rows per block.  Each cell: ubar = (b + sum_f c_f u_f)/D,
// u <- omega*ubar + (1-omega)*u.  The residual rows of the stopping rule are
// formed on the way: red rows of iterate k-1 are D(ubar - u^(k-1)), black rows
// of iterate k are D(1-omega)(ubar - u_old).
template <int COLOR>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs a)
{
    __shared__ double lds[4];
    __shared__ int flag;
    Ctrl* C = a.C;
    if (C->done) return;
    const Layout& L = a.L;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int ntm = (L.half + 63) >> 6;
    const int64_t ntr = (L.nrow_int + 3) >> 2;
    const int64_t sy = L.rs, sz = (int64_t)L.p2 * L.rs, st = (int64_t)L.p2 * L.p3 * L.rs;
    const int64_t cs = L.csplit;
    const double om = a.omega, om1 = 1.0 - a.omega;
    double acc = 0.0;
    for (TileWalk tw(ntm * ntr); tw.t < tw.end; tw.t += tw.step) {
        const int64_t tr = tw.t / ntm;
        const int tm = (int)(tw.t - tr * ntm);
        const int64_t r = tr * 4 + ty;
        const int m = tm * 64 + tx;
        if (r >= L.nrow_int) continue;
        const int j = (int)(r % L.n2) + 1;
        const int64_t r2 = r / L.n2;
        const int k = (int)(r2 % L.n3) + 1;
        const int l = (int)(r2 / L.n3) + 1;
        const int par = (COLOR + j + k + l) & 1;
        const int cnt = par ? (L.n1 + 1) >> 1 : L.n1 >> 1;
        if (m >= cnt) continue;
        const int64_t prow = ((int64_t)l * L.p3 + k) * L.p2 + j;
        const int64_t ui = prow * L.rs + L.xoff + m;
        const int64_t ci = r * L.rsc + m;
        const double c0 = a.coef[ci], c1 = a.coef[cs + ci], c2 = a.coef[2 * cs + ci], c3 = a.coef[3 * cs + ci];
        const double c4 = a.coef[4 * cs + ci], c5 = a.coef[5 * cs + ci], c6 = a.coef[6 * cs + ci], c7 = a.coef[7 * cs + ci];
        const double* uo = a.uoth;
        double s = a.rhs[ci];
        s += c0 * uo[ui - par] + c1 * uo[ui + 1 - par];
        s += c2 * uo[ui - sy] + c3 * uo[ui + sy];
        s += c4 * uo[ui - sz] + c5 * uo[ui + sz];
        s += c6 * uo[ui - st] + c7 * uo[ui + st];
        const double D = ((((((((1.0 + c0) + c1) + c2) + c3) + c4) + c5) + c6) + c7);
        const double ub = s / D;
        const double uold = a.uin[ui];
        a.uout[ui] = om * ub + om1 * uold;
        const double rres = COLOR == 0 ? D * (ub - uold) : D * om1 * (ub - uold);
        acc += rres * rres;
    }
    const double bs = block_sum(acc, lds);
    if (threadIdx.x == 0) a.part[blockIdx.x] = bs;
    if (COLOR == 1 || !a.check) return;
    if (!arrive_last(&C->arrive[1], gridDim.x, &flag)) return;
    const double Rr = sum_partials(a.part, gridDim.x, lds);
    const double Rb = sum_partials(a.part_other, gridDim.x, lds);
    if (threadIdx.x == 0) {
        const int kk = a.k - 1;
        const double R2 = Rb + Rr;
        const double R = sqrt(R2);
        C->rel_res = C->bn > 0.0 ? R / C->bn : R;
        if (!(R2 < INFINITY)) {
            C->status = SUBSURF4D_ENONFINITE;
            C->done = 1;
            C->iterations = kk;
            C->final_red = kk & 1;
        } else if (R <= C->tol * C->bn) {
            C->done = 1;
            C->iterations = kk;
            C->final_red = kk & 1;
        } else if (kk >= C->max_iter) {
            C->status = SUBSURF4D_NOT_CONVERGED;
            C->done = 1;
            C->iterations = kk;
            C->final_red = kk & 1;
        }
        C->arrive[1] = 0;
    }
}

// colour-split u -> interior of the padded u
__global__ __launch_bounds__(kBlock) void k_unsplit(Layout L, const double* ured0, const double* ured1,
                                                    const double* ublack, const Ctrl* C, double* u)
{
    const double* red = C->final_red ? ured1 : ured0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < L.nint; q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q % L.n1) + 1;
        const int64_t row = q / L.n1;
        const int j = (int)(row % L.n2) + 1;
        const int64_t r2 = row / L.n2;
        const int k = (int)(r2 % L.n3) + 1;
        const int l = (int)(r2 / L.n3) + 1;
        const int64_t prow = ((int64_t)l * L.p3 + k) * L.p2 + j;
        const int64_t us = prow * L.rs + L.xoff + ((i - 1) >> 1);
        const double v = ((i + j + k + l) & 1) ? ublack[us] : red[us];
        u[prow * L.p1 + i] = v;
    }
}

int sweep_grid(const Layout& L)
{
    const int64_t ntiles = (int64_t)((L.half + 63) >> 6) * ((L.nrow_int + 3) >> 2);
    return grid_for(ntiles, 1);
}

void fill_result(const Ctrl& hc, subsurf4d_result* res)
{
    if (!res) return;
    res->status = hc.status;
    res->iterations = hc.iterations;
    res->outer_iterations = hc.outer;
    res->reserved = 0;
    res->rel_residual = hc.rel_res;
    res->bnorm = hc.bn;
}

void effective_stop(const subsurf4d_step_params& sp, double* tol, int* max_iter)
{
    if (sp.fixed_iters > 0) { *tol = 0.0; *max_iter = sp.fixed_iters; }
    else { *tol = sp.tol; *max_iter = sp.max_iter; }
}

}  // namespace

int run_sor_loop(const WsPlan& P, const subsurf4d_step_params& sp, void* ws, hipStream_t s,
                 subsurf4d_result* res)
{
    const Layout& L = P.L;
    Ctrl* C = ws_ptr<Ctrl>(ws, P.ctrl);
    double* ured[2] = {ws_ptr<double>(ws, P.ured0), ws_ptr<double>(ws, P.ured1)};
    double* ublack = ws_ptr<double>(ws, P.ublack);
    const double* coef = ws_ptr<double>(ws, P.coef);
    const double* rhs = ws_ptr<double>(ws, P.rhs);
    double* pa = ws_ptr<double>(ws, P.part_a);
    double* pb = ws_ptr<double>(ws, P.part_b);
    double tol;
    int max_iter;
    effective_stop(sp, &tol, &max_iter);
    const int check_every = sp.check_every > 0 ? sp.check_every : 1;
    const int grid = sweep_grid(L);

    SweepArgs red{}, black{};
    red.L = black.L = L;
    red.omega = black.omega = sp.omega;
    red.C = black.C = C;
    red.coef = coef;
    red.rhs = rhs;
    black.coef = coef + 8 * L.csplit;
    black.rhs = rhs + L.csplit;
    red.part = pa;
    red.part_other = pb;
    black.part = pb;
    black.uin = black.uout = ublack;
    red.uoth = ublack;

    Ctrl hc;
    SS4_HIP(hipMemcpyAsync(&hc, C, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    SS4_HIP(hipStreamSynchronize(s));
    SweepTimer timer(s);
    int k = 1;
    int chunk = sp.iter_hint > 0 ? sp.iter_hint + 1 : 8;
    while (!hc.done) {
        timer.begin();
        for (int c = 0; c < chunk && k <= max_iter + 1; ++c, ++k) {
            red.k = k;
            red.uin = ured[(k - 1) & 1];
            red.uout = ured[k & 1];
            red.check = (k >= 2) && (((k - 1) % check_every == 0) || (k - 1 >= max_iter));
            k_sweep<0><<<grid, kBlock, 0, s>>>(red);
            if (k <= max_iter) {
                black.k = k;
                black.uoth = ured[k & 1];
                k_sweep<1><<<grid, kBlock, 0, s>>>(black);
            }
        }
        SS4_LAUNCHED("sweeps");
        timer.end();
        SS4_HIP(hipMemcpyAsync(&hc, C, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
        SS4_HIP(hipStreamSynchronize(s));
        timer.collect();
        if (k > max_iter + 1 && !hc.done) {
            set_error("internal: iteration ended without a decision");
            return SUBSURF4D_EDEVICE;
        }
        chunk = chunk < 64 ? chunk * 2 : 64;
    }
    fill_result(hc, res);
    // launches that did work: red k = 1..K+1 (the last one tests iterate K), black k = 1..K
    timer.account(hc.iterations > 0 || hc.done ? 2 * (int64_t)hc.iterations + (hc.iterations > 0 ? 1 : 0) : 0,
                  (int64_t)hc.iterations * L.nint);
    if (hc.status == SUBSURF4D_ENONFINITE) {
        set_error("non-finite residual in the SOR solve");
        return SUBSURF4D_ENONFINITE;
    }
    return 0;
}

int run_unsplit(const WsPlan& P, double* u, void* ws, hipStream_t s)
{
    const Layout& L = P.L;
    k_unsplit<<<grid_for(L.nint), kBlock, 0, s>>>(L, ws_ptr<double>(ws, P.ured0), ws_ptr<double>(ws, P.ured1),
                                                  ws_ptr<double>(ws, P.ublack), ws_ptr<Ctrl>(ws, P.ctrl), u);
    SS4_LAUNCHED("unsplit");
    return 0;
}

int run_assemble_export(const Layout& L, double h, const double* G, const double* u,
                        const subsurf4d_step_params& sp, double* coef, double* b, hipStream_t s)
{
    AsmArgs a{};
    a.L = L;
    a.th2 = sp.tau / (h * h);
    a.eps2 = sp.eps * sp.eps;
    a.inv_h = 1.0 / h;
    a.G = G;
    a.w = u;
    a.coef_nat = coef;
    a.b_nat = b;
    k_assemble<kNatural><<<grid_for(L.npad), kBlock, 0, s>>>(a);
    SS4_LAUNCHED("assemble (export)");
    return 0;
}

int run_step(const WsPlan& P, double h, const double* G, const subsurf4d_centre* centres, int nc,
             const int32_t* owner, double* u, const subsurf4d_step_params& sp, subsurf4d_result* res,
             void* ws, hipStream_t s)
{
    const Layout& L = P.L;
    Ctrl* C = ws_ptr<Ctrl>(ws, P.ctrl);
    int rc;
    if (sp.precision == SUBSURF4D_MIXED) {
        rc = run_mixed_solve(P, h, G, u, sp, res, ws, s);
        if (rc < 0) return rc;
    } else {
        double tol;
        int max_iter;
        effective_stop(sp, &tol, &max_iter);
        k_ctrl_init<<<1, 64, 0, s>>>(C, tol, max_iter);
        AsmArgs a{};
        a.L = L;
        a.th2 = sp.tau / (h * h);
        a.eps2 = sp.eps * sp.eps;
        a.inv_h = 1.0 / h;
        a.G = G;
        a.w = u;
        a.ured0 = ws_ptr<double>(ws, P.ured0);
        a.ured1 = ws_ptr<double>(ws, P.ured1);
        a.ublack = ws_ptr<double>(ws, P.ublack);
        a.coef = ws_ptr<double>(ws, P.coef);
        a.rhs = ws_ptr<double>(ws, P.rhs);
        a.part_a = ws_ptr<double>(ws, P.part_a);
        a.part_b = ws_ptr<double>(ws, P.part_b);
        a.C = C;
        k_assemble<kSplit><<<grid_for(L.npad), kBlock, 0, s>>>(a);
        SS4_LAUNCHED("assemble");
        rc = run_sor_loop(P, sp, ws, s, res);
        if (rc < 0) return rc;
        rc = run_unsplit(P, u, ws, s);
        if (rc < 0) return rc;
    }
    if (sp.rescale && nc > 0) {
        const int r2 = run_rescale(P, centres, nc, sp.ball_r, owner, u, ws, s);
        if (r2 < 0) return r2;
    }
    SS4_HIP(hipStreamSynchronize(s));
    return res ? res->status : 0;
}

int run_solve(const WsPlan& P, const double* coef, const double* b, double* u,
              const subsurf4d_step_params& sp, subsurf4d_result* res, void* ws, hipStream_t s)
{
    const Layout& L = P.L;
    Ctrl* C = ws_ptr<Ctrl>(ws, P.ctrl);
    double tol;
    int max_iter;
    effective_stop(sp, &tol, &max_iter);
    k_ctrl_init<<<1, 64, 0, s>>>(C, tol, max_iter);
    k_load_system<<<grid_for(L.npad), kBlock, 0, s>>>(L, coef, b, u, ws_ptr<double>(ws, P.ured0),
                                                      ws_ptr<double>(ws, P.ured1), ws_ptr<double>(ws, P.ublack),
                                                      ws_ptr<double>(ws, P.coef), ws_ptr<double>(ws, P.rhs),
                                                      ws_ptr<double>(ws, P.part_a), ws_ptr<double>(ws, P.part_b), C);
    SS4_LAUNCHED("load system");
    int rc = run_sor_loop(P, sp, ws, s, res);
    if (rc < 0) return rc;
    rc = run_unsplit(P, u, ws, s);
    if (rc < 0) return rc;
    SS4_HIP(hipStreamSynchronize(s));
    return res ? res->status : 0;
}

}  // namespace ss4
