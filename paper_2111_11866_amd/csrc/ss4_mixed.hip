// Mixed-precision solve of one step's system: FP64 iterative refinement
// around FP32 red-black SOR sweeps on BF16-stored, diagonal-scaled
// coefficients.
//
//   x = u^{resc;n-1}                                      (FP64, colour-split)
//   repeat:  r = b - A x            FP64 operator, FP64 arithmetic
//            stop if ||r||_2 <= refine_tol ||b||_2
//            solve (I - C') d = r/D approximately by `inner_sweeps` red-black
//              SOR iterations in FP32, C' = off-diagonal coefficients / D in BF16
//            x += d                                        (FP64)
//
// The residual always uses the FP64 operator, so the refinement converges to
// the FP64 system's solution; the BF16 operator only steers the corrections.
#include <cmath>

#include "ss4_internal.hpp"

namespace ss4 {
namespace {

struct MxArgs {
    Layout L;
    const double* coef;   // FP64 tiled coefficients + rhs (both colours)
    const uint4* c16;     // BF16 records (both colours)
    float* rf;            // scaled FP32 residual r/D, record index
    double* xr;           // x, red colour-split (padded rows, ghosts = Dirichlet data)
    double* xb;           // x, black
    float* dr;            // correction d, red (ghost slots stay 0)
    float* db;            // correction d, black
    double* part;
    Ctrl* C;
    float omega;
    int pass;             // refinement passes completed before this residual
    int max_outer;
};

__device__ __forceinline__ uint4 ld16_stream(const uint4* p)
{
    typedef unsigned int u4v __attribute__((ext_vector_type(4)));
    const u4v v = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

// FP64 residual of x for every interior cell of both colours; writes r/D in
// FP32; the last block applies the refinement stopping rule.
__global__ __launch_bounds__(kBlock) void k_mx_residual(MxArgs a)
{
    __shared__ double lds[4];
    __shared__ int flag;
    if (a.C->done) return;      // enqueue-only calls: a pass after the decision
    const Layout& L = a.L;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int ntm = (L.half + 63) >> 6;
    const int njb = (L.n2 + 3) >> 2;
    const int64_t ncol = (int64_t)ntm * njb * L.n3;
    const int64_t sy = L.rs, sz = (int64_t)L.p2 * L.rs, st = (int64_t)L.p2 * L.p3 * L.rs;
    double acc = 0.0;
    // a block owns a 64-slot x 4-row column tile at one z and walks the
    // frames for both colours; the other colour's t-neighbours stay in
    // registers (tiles dealt slot-tile fastest, then z, as the sweeps)
    for (TileWalk tw(ncol); tw.t < tw.end; tw.t += tw.step) {
        const int mt = (int)(tw.t % ntm);
        const int64_t t2 = tw.t / ntm;
        const int k = (int)(t2 % L.n3) + 1;
        const int jb = (int)(t2 / L.n3);
        const int j = jb * 4 + ty + 1;
        const int m = mt * 64 + tx;
        if (j > L.n2 || m >= L.half) continue;
        const int64_t ub = ((int64_t)k * L.p2 + j) * L.rs + L.xoff + m;
        const int64_t rb = (int64_t)(k - 1) * L.n2 + (j - 1);
        for (int colour = 0; colour < 2; ++colour) {
            const double* own = colour ? a.xb : a.xr;
            const double* oth = colour ? a.xr : a.xb;
            double Bm = oth[ub];
            double Bc = oth[ub + st];
            for (int l = 1; l <= L.n4; ++l) {
                const int64_t ui = ub + (int64_t)l * st;
                const double Bp = oth[ui + st];
                const int par = (colour + j + k + l) & 1;
                const int cnt = par ? (L.n1 + 1) >> 1 : L.n1 >> 1;
                if (m < cnt) {
                    const int64_t r = rb + (int64_t)(l - 1) * L.n3 * L.n2;
                    const double* cf = a.coef + ctile(L, colour, r, m);
                    // touched once per residual: non-temporal, so the neighbour rows stay in L2
                    auto ld = [](const double* p) { return __builtin_nontemporal_load(p); };
                    const double c0 = ld(cf), c1 = ld(cf + kTileSlots), c2 = ld(cf + 2 * kTileSlots);
                    const double c3 = ld(cf + 3 * kTileSlots), c4 = ld(cf + 4 * kTileSlots);
                    const double c5 = ld(cf + 5 * kTileSlots), c6 = ld(cf + 6 * kTileSlots);
                    const double c7 = ld(cf + 7 * kTileSlots);
                    const double xo = oth[par ? ui - 1 : ui + 1];
                    double s = ld(cf + 8 * kTileSlots);
                    s += c0 * (par ? xo : Bc) + c1 * (par ? Bc : xo);
                    s += c2 * oth[ui - sy] + c3 * oth[ui + sy];
                    s += c4 * oth[ui - sz] + c5 * oth[ui + sz];
                    s += c6 * Bm + c7 * Bp;
                    const double D = ((((((((1.0 + c0) + c1) + c2) + c3) + c4) + c5) + c6) + c7);
                    const double res = s - D * ld(own + ui);
                    acc += res * res;
                    a.rf[mrec(L, colour, r, m)] = (float)(res / D);
                }
                Bm = Bc;
                Bc = Bp;
            }
        }
    }
    const double bs = block_sum(acc, lds);
    if (threadIdx.x == 0) a.part[blockIdx.x] = bs;
    if (!arrive_last(&a.C->arrive[2], gridDim.x, &flag)) return;
    const double R2 = sum_partials(a.part, gridDim.x, lds);
    if (threadIdx.x == 0) {
        Ctrl* C = a.C;
        const double R = sqrt(R2);
        C->rel_res = C->bn > 0.0 ? R / C->bn : R;
        C->outer = a.pass;
        if (!(R2 < INFINITY)) { C->status = SUBSURF4D_ENONFINITE; C->done = 1; }
        else if (R <= C->tol * C->bn) { C->status = SUBSURF4D_OK; C->done = 1; }
        else if (a.pass >= a.max_outer) { C->status = SUBSURF4D_NOT_CONVERGED; C->done = 1; }
        C->arrive[2] = 0;
    }
}

// One relaxed update of the scaled correction system.
__device__ __forceinline__ float mx_cell(uint4 w, float rhs, float xl, float xr, float ym, float yp, float zm, float zp,
                                         float tm, float tp, float om, float om1, float old)
{
    float s = rhs;
    s += bf16_lo(w.x) * xl + bf16_hi(w.x) * xr;
    s += bf16_lo(w.y) * ym + bf16_hi(w.y) * yp;
    s += bf16_lo(w.z) * zm + bf16_hi(w.z) * zp;
    s += bf16_lo(w.w) * tm + bf16_hi(w.w) * tp;
    return om * s + om1 * old;
}

// FP32 red-black half-sweep on the scaled correction system, frame-marching
// form (as the FP64 sweep): d <- omega*(r/D + sum_f c'_f d_f) + (1-omega)*d.
// FIRST: the first iteration of a refinement pass, which starts from d = 0.
// Its red half-sweep is then d = omega*r/D (no coefficient or neighbour
// reads) and its black half-sweep takes the old d as 0 without reading it;
// both give the bits of the general form on a zero d, so no pass needs d
// cleared beforehand.
template <int COLOR, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_mx_sweep(MxArgs a)
{
    if (a.C->done) return;
    const Layout& L = a.L;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int ntm = (L.half + 63) >> 6;
    const int njb = (L.n2 + 3) >> 2;
    const int64_t ncol = (int64_t)ntm * njb * L.n3;
    const int64_t sy = L.rs, sz = (int64_t)L.p2 * L.rs, st = (int64_t)L.p2 * L.p3 * L.rs;
    const int last_slot = L.n1 >> 1;
    const float om = a.omega, om1 = 1.0f - a.omega;
    float* own = COLOR ? a.db : a.dr;
    const float* __restrict__ oth = COLOR ? a.dr : a.db;
    for (TileWalk tw(ncol); tw.t < tw.end; tw.t += tw.step) {
        const int mt = (int)(tw.t % ntm);                // slot-tile fastest, then k (as the FP64 sweep)
        const int64_t t2 = tw.t / ntm;
        const int k = (int)(t2 % L.n3) + 1;
        const int jb = (int)(t2 / L.n3);
        const int j = jb * 4 + ty + 1;
        const int m = mt * 64 + tx;
        const bool jok = j <= L.n2;
        const bool sok = jok && m <= last_slot;
        const int64_t ub = ((int64_t)k * L.p2 + j) * L.rs + L.xoff + m;
        const int64_t rb = (int64_t)(k - 1) * L.n2 + (j - 1);
        if constexpr (FIRST && COLOR == 0) {
            if (!jok) continue;
            for (int l = 1; l <= L.n4; ++l) {
                const int par = (COLOR + j + k + l) & 1;
                const int cnt = par ? (L.n1 + 1) >> 1 : L.n1 >> 1;
                if (m < cnt) {
                    const int64_t q = mrec(L, COLOR, rb + (int64_t)(l - 1) * L.n3 * L.n2, m);
                    own[ub + (int64_t)l * st] = om * __builtin_nontemporal_load(a.rf + q);
                }
            }
            continue;
        }
        float Bm = sok ? oth[ub] : 0.0f;
        float Bc = sok ? oth[ub + st] : 0.0f;
        for (int l = 1; l <= L.n4; ++l) {
            const int64_t ui = ub + (int64_t)l * st;
            const float Bp = sok ? oth[ui + st] : 0.0f;
            const int par = (COLOR + j + k + l) & 1;
            float left = __shfl_up(Bc, 1);
            float right = __shfl_down(Bc, 1);
            if (jok) {
                if (tx == 0 && par) left = oth[ui - 1];
                if (tx == 63 && !par && m + 1 <= last_slot) right = oth[ui + 1];
                const int cnt = par ? (L.n1 + 1) >> 1 : L.n1 >> 1;
                if (m < cnt) {
                    const int64_t q = mrec(L, COLOR, rb + (int64_t)(l - 1) * L.n3 * L.n2, m);
                    const uint4 w = ld16_stream(a.c16 + q);
                    const float rhs = __builtin_nontemporal_load(a.rf + q);
                    own[ui] = mx_cell(w, rhs, par ? left : Bc, par ? Bc : right, oth[ui - sy], oth[ui + sy],
                                      oth[ui - sz], oth[ui + sz], Bm, Bp, om, om1, FIRST ? 0.0f : own[ui]);
                }
            }
            Bm = Bc;
            Bc = Bp;
        }
    }
}

// x += d on every interior cell of both colours (the next pass's first
// iteration does not read d).
__global__ __launch_bounds__(kBlock) void k_mx_update(MxArgs a)
{
    if (a.C->done) return;
    const Layout& L = a.L;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int ntm = (L.half + 63) >> 6;
    const int64_t rows = 2 * L.nrow_int;
    const int64_t ntr = (rows + 3) >> 2;
    for (TileWalk tw(ntm * ntr); tw.t < tw.end; tw.t += tw.step) {
        const int64_t tr = tw.t / ntm;
        const int tm = (int)(tw.t - tr * ntm);
        const int64_t rr = tr * 4 + ty;
        if (rr >= rows) continue;
        const int colour = rr >= L.nrow_int ? 1 : 0;
        const int64_t r = rr - colour * L.nrow_int;
        const int m = tm * 64 + tx;
        const int j = (int)(r % L.n2) + 1;
        const int64_t r2 = r / L.n2;
        const int k = (int)(r2 % L.n3) + 1;
        const int l = (int)(r2 / L.n3) + 1;
        const int par = (colour + j + k + l) & 1;
        const int cnt = par ? (L.n1 + 1) >> 1 : L.n1 >> 1;
        if (m >= cnt) continue;
        const int64_t ui = (((int64_t)l * L.p3 + k) * L.p2 + j) * L.rs + L.xoff + m;
        double* x = colour ? a.xb : a.xr;
        float* d = colour ? a.db : a.dr;
        x[ui] += (double)d[ui];
    }
}

__global__ void k_fill_f32(float* a, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        a[q] = 0.0f;
}

}  // namespace

int run_mixed_solve(const WsPlan& P, double h, const double* G, const double* w, const double* ub,
                    const subsurf4d_step_params& sp, subsurf4d_result* res, void* ws, hipStream_t s)
{
    const Layout& L = P.L;
    Ctrl* C = ws_ptr<Ctrl>(ws, P.ctrl);
    const int m = sp.inner_sweeps;
    const int max_outer = sp.max_iter / m > 1 ? sp.max_iter / m : 1;
    MxArgs a{};
    a.L = L;
    a.coef = ws_ptr<double>(ws, P.coef);
    a.c16 = ws_ptr<uint4>(ws, P.coef16);
    a.rf = ws_ptr<float>(ws, P.rf32);
    a.xr = ws_ptr<double>(ws, P.ured0);
    a.xb = ws_ptr<double>(ws, P.ublack);
    a.dr = ws_ptr<float>(ws, P.dred);
    a.db = ws_ptr<float>(ws, P.dblack);
    a.part = ws_ptr<double>(ws, P.part_a);
    a.C = C;
    a.omega = (float)sp.omega;
    a.max_outer = max_outer;

    k_ctrl_init<<<1, 64, 0, s>>>(C, sp.refine_tol, max_outer);
    int rc = launch_assembly(P, h, G, w, ub, sp, ws_ptr<void>(ws, P.coef16), ws, s);
    if (rc < 0) return rc;
    k_fill_f32<<<grid_for(L.usplit), kBlock, 0, s>>>(a.dr, L.usplit);
    k_fill_f32<<<grid_for(L.usplit), kBlock, 0, s>>>(a.db, L.usplit);
    SS4_LAUNCHED("mixed: init");

    const int64_t row_tiles = (int64_t)((L.half + 63) >> 6) * ((2 * L.nrow_int + 3) >> 2);
    const int grid_rows = grid_for(row_tiles, 1);
    const int grid_res = resident_grid(reinterpret_cast<const void*>(&k_mx_residual));
    auto residual = [&]() { k_mx_residual<<<grid_res, kBlock, 0, s>>>(a); };
    const int64_t ncol = (int64_t)((L.half + 63) >> 6) * ((L.n2 + 3) >> 2) * L.n3;
    // one cell per lane: two cells per lane (as the FP64 sweep) measured slower
    // for the FP32 correction, in two designs (3.36 vs 4.13 TB/s on the
    // 512x512x96x16 volume; a tile-per-wave form with contiguous 2 KB record
    // runs and 8-byte d accesses, same bits: 165.7 vs 162.1 ms per step)
    // three quarters of the resident grid: on the 512x512x96x16 volume the
    // concurrent window of an XCD is then 48 z-planes x 4 slot tiles, half a
    // row of tiles (1.493 ms per half-sweep against 1.535 at one half, 1.52-1.68
    // at 60-125% except 150%, 1.507, a whole row); same iterate for any grid
    int res_g = (int)((int64_t)resident_grid(reinterpret_cast<const void*>(&k_mx_sweep<0, false>)) *
                      sweep_grid_percent(75) / 100);
    if (res_g > kGridCap) res_g = kGridCap;   // the per-block partial arrays hold kGridCap entries
    const int grid_cols = (int)(((ncol < res_g ? ncol : res_g) + kXcd - 1) / kXcd * kXcd);

    auto enqueue_sweeps = [&](int mm) {
        k_mx_sweep<0, true><<<grid_cols, kBlock, 0, s>>>(a);
        k_mx_sweep<1, true><<<grid_cols, kBlock, 0, s>>>(a);
        for (int it = 1; it < mm; ++it) {
            k_mx_sweep<0, false><<<grid_cols, kBlock, 0, s>>>(a);
            k_mx_sweep<1, false><<<grid_cols, kBlock, 0, s>>>(a);
        }
    };
    if (sp.flags & SUBSURF4D_FLAG_ASYNC) {
        // enqueue-only: every pass up to the cap; the kernels of a pass after
        // the residual's decision return at once
        for (int pass = 0; pass <= max_outer; ++pass) {
            a.pass = pass;
            residual();
            if (pass == max_outer) break;
            enqueue_sweeps(m);
            k_mx_update<<<grid_rows, kBlock, 0, s>>>(a);
        }
        SS4_LAUNCHED("mixed: refinement passes");
        return 0;
    }

    Ctrl hc;
    SS4_HIP(hipMemcpyAsync(&hc, C, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    SS4_HIP(hipStreamSynchronize(s));
    SweepTimer timer(s);
    const bool shorten = (sp.flags & SUBSURF4D_FLAG_SHORT_LAST_PASS) != 0;
    int pass = 0;
    int64_t sweeps = 0;       // FP32 red-black iterations enqueued
    double prev_res = 0.0;    // relative FP64 residual before the previous pass
    int prev_m = 0;           // that pass's iterations
    while (!hc.done) {
        a.pass = pass;
        residual();
        SS4_LAUNCHED("mixed: residual");
        SS4_HIP(hipMemcpyAsync(&hc, C, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
        SS4_HIP(hipStreamSynchronize(s));
        if (hc.done) break;
        int mm = m;
        if (shorten && pass >= 2 && prev_res > 0.0 && hc.rel_res > 0.0 && hc.rel_res < prev_res &&
            sp.refine_tol < hc.rel_res) {
            // per-iteration contraction over the previous pass, and the
            // iterations it predicts for reaching refine_tol
            const double rho = pow(hc.rel_res / prev_res, 1.0 / prev_m);
            const double need = log(sp.refine_tol / hc.rel_res) / log(rho);
            if (need < (double)m) {
                const int pred = (int)ceil(1.25 * need) + 1;
                if (pred < mm) mm = pred;
            }
        }
        prev_res = hc.rel_res;
        prev_m = mm;
        timer.begin();
        enqueue_sweeps(mm);
        timer.end();
        k_mx_update<<<grid_rows, kBlock, 0, s>>>(a);
        SS4_LAUNCHED("mixed: inner sweeps");
        sweeps += mm;
        ++pass;
        if (timer.end_event()) {
            SS4_HIP(hipEventSynchronize(timer.end_event()));
            timer.collect();
        }
    }
    timer.account(2 * sweeps, sweeps * L.nint);
    res->status = hc.status;
    res->iterations = (int32_t)sweeps;
    res->outer_iterations = hc.outer;
    res->reserved = 0;
    res->rel_residual = hc.rel_res;
    res->bnorm = hc.bn;
    if (hc.status == SUBSURF4D_ENONFINITE) {
        set_error("non-finite residual in the mixed-precision solve");
        return SUBSURF4D_ENONFINITE;
    }
    return 0;
}

}  // namespace ss4
