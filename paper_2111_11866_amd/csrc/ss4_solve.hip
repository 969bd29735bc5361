// Time-step kernels: assembly of the finite-volume system from
// reduced-diamond-cell face gradients (Sec. 3.2.2, the uniform-h system with
// A_eps and A_eps-bar), red-black SOR half-sweeps with the residual norm fused
// in, and the host driver of the iteration.
#include <cmath>
#include <cstdlib>

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
    const double* w;  // padded u^{resc;n-1} (its ghosts feed the boundary-face gradients)
    const double* ub; // padded; ghost layer = Dirichlet data of the new level (== w when not separate)
    double* ured0;
    double* ured1;
    double* ublack;
    double* coef;     // tiled coefficient + rhs block, both colours
    uint4* coef16;    // optional: normalised BF16 coefficient records (mixed precision)
    double* coef_nat; // interior x 8
    double* b_nat;    // interior
    double* part_a;
    double* part_b;
    Ctrl* C;
};

// Per-block partials of ||b||^2 and of the initial residual, and (last block)
// the decision on iterate 0.
__device__ __forceinline__ void assembly_decide(const AsmArgs& a, double acc_b, double acc_r, double* lds, int* flagp)
{
    int& flag = *flagp;
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

// Coefficients, right-hand side and residual of the initial iterate of one
// interior cell p = (i,j,k,l) from the 33-point neighbourhood of w and G on
// its 8 faces; the colour-split tiles (MODE kSplit) or the natural arrays
// (kNatural) receive them.  Shared by both assembly kernels, so the
// coefficients do not depend on the visiting order.
template <int MODE, typename WAt, typename GAt>
__device__ __forceinline__ void assemble_cell(const AsmArgs& a, int64_t p, int i, int j, int k, int l, int colour,
                                              int m, WAt&& wat, GAt&& gat, double& acc_b, double& acc_r)
{
    const Layout& L = a.L;
    const int64_t s1 = 1, s2 = L.p1, s3 = (int64_t)L.p1 * L.p2, s4 = s3 * L.p3;
    const int64_t sd[4] = {s1, s2, s3, s4};
    const int idx[4] = {i, j, k, l};
    const int nn[4] = {L.n1, L.n2, L.n3, L.n4};
    // w at p + o, o a sum of at most two signed unit offsets (axis, sign)
    auto w1 = [&](int d, int sg) {
        return wat(d == 0 ? sg : 0, d == 1 ? sg : 0, d == 2 ? sg : 0, d == 3 ? sg : 0);
    };
    auto w2 = [&](int d, int sd_, int t, int st) {
        return wat((d == 0 ? sd_ : 0) + (t == 0 ? st : 0), (d == 1 ? sd_ : 0) + (t == 1 ? st : 0),
                   (d == 2 ? sd_ : 0) + (t == 2 ? st : 0), (d == 3 ? sd_ : 0) + (t == 3 ? st : 0));
    };
    const double w0 = wat(0, 0, 0, 0);
    // face neighbours
    double wm[4], wp[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) { wm[d] = w1(d, -1); wp[d] = w1(d, 1); }
    double q[8];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const double gnm = (w0 - wm[d]) * a.inv_h;   // normal, -e_d face
        const double gnp = (wp[d] - w0) * a.inv_h;   // normal, +e_d face
        double qm = gnm * gnm, qp = gnp * gnp;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t == d) continue;
            const double wpt = wp[t], wmt = wm[t];
            const double dm_pt = w2(d, -1, t, 1), dm_mt = w2(d, -1, t, -1);
            const double dp_pt = w2(d, 1, t, 1), dp_mt = w2(d, 1, t, -1);
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
        const double gm = gat(d, 0);     // face -e_d: G_d of p - e_d
        const double gp = gat(d, 1);     // face +e_d: G_d of p
        c[2 * d] = scale * gm / sqrt(a.eps2 + q[2 * d]);
        c[2 * d + 1] = scale * gp / sqrt(a.eps2 + q[2 * d + 1]);
    }
    double D = 1.0;
#pragma unroll
    for (int f = 0; f < 8; ++f) D += c[f];
    // right-hand side and residual of the initial iterate: Dirichlet
    // neighbours take the new level's data
    double bfull = w0, off = 0.0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const double vm = idx[d] == 1 ? a.ub[p - sd[d]] : wm[d];
        const double vp = idx[d] == nn[d] ? a.ub[p + sd[d]] : wp[d];
        off += c[2 * d] * vm + c[2 * d + 1] * vp;
        if (idx[d] == 1) bfull += c[2 * d] * vm;
        if (idx[d] == nn[d]) bfull += c[2 * d + 1] * vp;
    }
    const double r0 = (w0 + off) - D * w0;
    acc_b += bfull * bfull;
    acc_r += r0 * r0;
    const int64_t irow = ((int64_t)(l - 1) * L.n3 + (k - 1)) * L.n2 + (j - 1);
    if (MODE == kSplit) {
        const int64_t ci = ctile(L, colour, irow, m);
#pragma unroll
        for (int f = 0; f < 8; ++f) a.coef[ci + f * kTileSlots] = c[f];
        a.coef[ci + 8 * kTileSlots] = w0;
        if (a.coef16) {
            const double inv = 1.0 / D;
            uint32_t h[8];
#pragma unroll
            for (int f = 0; f < 8; ++f) h[f] = bf16_bits((float)(c[f] * inv));
            a.coef16[mrec(L, colour, irow, m)] =
                make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
        }
    } else {
        const int64_t qi = irow * L.n1 + (i - 1);
#pragma unroll
        for (int f = 0; f < 8; ++f) a.coef_nat[qi * 8 + f] = c[f];
        a.b_nat[qi] = bfull;
    }
}

// One thread per padded cell (flat order): ghost cells only copy the new
// level's Dirichlet value into the colour-split u; interior cells assemble.
// Used for the natural-layout export.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_assemble(AsmArgs a)
{
    __shared__ double lds[4];
    __shared__ int flag;
    const Layout& L = a.L;
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
        const bool inside = i >= 1 && i <= L.n1 && j >= 1 && j <= L.n2 && k >= 1 && k <= L.n3 && l >= 1 && l <= L.n4;
        if (MODE == kSplit) {
            const double v0 = inside ? w0 : a.ub[p];
            const int64_t us = prow * L.rs + L.xoff + m;
            if (colour == 0) { a.ured0[us] = v0; a.ured1[us] = v0; }
            else a.ublack[us] = v0;
        }
        if (!inside) continue;
        const int64_t s2 = L.p1, s3 = (int64_t)L.p1 * L.p2, s4 = s3 * L.p3;
        const int64_t sd[4] = {1, s2, s3, s4};
        assemble_cell<MODE>(
            a, p, i, j, k, l, colour, m,
            [&](int di, int dj, int dk, int dl) { return a.w[p + di + dj * s2 + dk * s3 + dl * s4]; },
            [&](int d, int plus) { return a.G[(int64_t)d * L.npad + p - (plus ? 0 : sd[d])]; }, acc_b, acc_r);
    }
    if (MODE != kSplit) return;
    assembly_decide(a, acc_b, acc_r, lds, &flag);
}

// Assembly for the solver, frame-marching with the 33-point neighbourhood
// staged in LDS: a block owns a column tile of 64 interior x-cells x 4
// y-rows at one z and walks the frames l = 1..N4.  Per frame it loads the
// 3 planes (z-1, z, z+1) x 6 rows (y-1 .. y+4) x 66 x-cells of frame l+1
// into a ring of three frame slots, so every w value comes from LDS and each
// frame's slab is read from memory once per block.  The t-face G of the frame
// below is kept in a register from the previous frame.  Tiles of one XCD are
// consecutive (x-tile fastest, then z), so the neighbour planes a block loads
// are loaded by the blocks beside it at about the same time (L2 hits).  Ghost
// cells are written by k_ghost_split.
constexpr int kAx = 66, kAy = 6, kAz = 3;                  // slab: x with halo, y rows with halo, z planes
constexpr int kSlab = kAx * kAy * kAz;                     // doubles per frame slot

template <bool PREFETCH>
__global__ __launch_bounds__(kBlock) void k_assemble_cols(AsmArgs a)
{
    __shared__ double lds[4];
    __shared__ int flag;
    __shared__ double slab[3][kSlab];
    const Layout& L = a.L;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int nxt = (L.n1 + 63) >> 6;
    const int njb = (L.n2 + 3) >> 2;
    const int64_t ncol = (int64_t)nxt * njb * L.n3;
    const int64_t s2 = L.p1, s3 = (int64_t)L.p1 * L.p2, s4 = s3 * L.p3;
    double acc_b = 0.0, acc_r = 0.0;
    for (TileWalk tw(ncol); tw.t < tw.end; tw.t += tw.step) {
        const int xt = (int)(tw.t % nxt);
        const int64_t t2 = tw.t / nxt;
        const int k = (int)(t2 % L.n3) + 1;
        const int jb = (int)(t2 / L.n3);
        const int x0 = xt * 64 + 1, j0 = jb * 4 + 1;
        const int i = x0 + tx;
        const int j = j0 + ty;
        const bool active = i <= L.n1 && j <= L.n2;
        // slab of frame lf: padded x0-1 .. x0+64, y j0-1 .. j0+4, z k-1 .. k+1; this
        // thread's share (entries threadIdx.x + r*kBlock) goes to registers
        // first, so the loads of frame l+2 are in flight while frame l is
        // assembled, and then to the ring slot lf % 3
        constexpr int kPer = (kSlab + kBlock - 1) / kBlock;
        double pf[kPer];
        auto source = [&](int q) -> int64_t {     // offset within a frame, -1: outside the padded box
            const int pz = q / (kAx * kAy);
            const int rem = q - pz * (kAx * kAy);
            const int ry = rem / kAx;
            const int cx = rem - ry * kAx;
            const int ii = x0 - 1 + cx, jj = j0 - 1 + ry, kk = k - 1 + pz;
            return (q < kSlab && ii < L.p1 && jj < L.p2) ? (int64_t)kk * s3 + (int64_t)jj * s2 + ii : -1;
        };
        auto fetch = [&](int lf) {
            const double* fw = a.w + (int64_t)lf * s4;
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                const int64_t o = source(threadIdx.x + r * kBlock);
                pf[r] = o >= 0 ? fw[o] : 0.0;
            }
        };
        auto store = [&](int lf) {
            double* dst = slab[lf % 3];
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                const int q = threadIdx.x + r * kBlock;
                if (q < kSlab) dst[q] = pf[r];
            }
        };
        auto load = [&](int lf) {               // without prefetch: straight from memory to LDS
            double* dst = slab[lf % 3];
            const double* fw = a.w + (int64_t)lf * s4;
            for (int q = threadIdx.x; q < kSlab; q += kBlock) {
                const int64_t o = source(q);
                dst[q] = o >= 0 ? fw[o] : 0.0;
            }
        };
        __syncthreads();                 // the previous tile's last frame is no longer read
        load(0);
        load(1);
        if (PREFETCH) fetch(2);
        double gt_below = active ? a.G[3 * L.npad + ((int64_t)k * L.p2 + j) * L.p1 + i] : 0.0;   // G_t of frame 0
        for (int l = 1; l <= L.n4; ++l) {
            if (PREFETCH) store(l + 1);
            else load(l + 1);
            __syncthreads();
            if (PREFETCH && l + 2 <= L.n4 + 1) fetch(l + 2);
            if (active) {
                const int64_t prow = ((int64_t)l * L.p3 + k) * L.p2 + j;
                const int64_t p = prow * L.p1 + i;
                const int colour = (i + j + k + l) & 1;
                const int m = (i - 1) >> 1;
                const double w0 = slab[l % 3][(1 * kAy + ty + 1) * kAx + tx + 1];
                const int64_t us = prow * L.rs + L.xoff + m;
                if (colour == 0) { a.ured0[us] = w0; a.ured1[us] = w0; }
                else a.ublack[us] = w0;
                const double gt_here = a.G[3 * L.npad + p];
                const int sl[3] = {(l + 2) % 3, l % 3, (l + 1) % 3};      // slots of frames l-1, l, l+1
                assemble_cell<kSplit>(
                    a, p, i, j, k, l, colour, m,
                    [&](int di, int dj, int dk, int dl) {
                        return slab[sl[dl + 1]][((dk + 1) * kAy + ty + 1 + dj) * kAx + tx + 1 + di];
                    },
                    [&](int d, int plus) {
                        if (d == 3) return plus ? gt_here : gt_below;
                        const int64_t o = d == 0 ? 1 : (d == 1 ? s2 : s3);
                        return a.G[(int64_t)d * L.npad + p - (plus ? 0 : o)];
                    },
                    acc_b, acc_r);
                gt_below = gt_here;
            }
            __syncthreads();             // frame l-1's slot is refilled with frame l+2 next
        }
    }
    assembly_decide(a, acc_b, acc_r, lds, &flag);
}

// The ghost layer of the colour-split u: the new level's Dirichlet data.  One
// wave per padded row: rows in the ghost layer copy every cell, interior rows
// their two x-ghosts.
__global__ __launch_bounds__(kBlock) void k_ghost_split(Layout L, const double* __restrict__ ub, double* ured0,
                                                        double* ured1, double* ublack)
{
    const int tx = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t prow = wave; prow < L.nrow_pad; prow += nwaves) {
        const int j = (int)(prow % L.p2);
        const int64_t t2 = prow / L.p2;
        const int k = (int)(t2 % L.p3);
        const int l = (int)(t2 / L.p3);
        const bool ghost_row = j == 0 || j > L.n2 || k == 0 || k > L.n3 || l == 0 || l > L.n4;
        const int step = ghost_row ? 64 : L.p1;
        for (int i = ghost_row ? tx : (tx == 0 ? 0 : (tx == 1 ? L.n1 + 1 : L.p1)); i < L.p1; i += step) {
            const int64_t p = prow * L.p1 + i;
            const int m = (i - 1) >> 1;
            const int64_t us = prow * L.rs + L.xoff + m;
            const double v = ub[p];
            if (((i + j + k + l) & 1) == 0) { ured0[us] = v; ured1[us] = v; }
            else ublack[us] = v;
        }
    }
}

// Load an externally given system (natural layout, Dirichlet terms in b) into
// the colour-split arrays; ghost slots of u are 0 so they contribute nothing.
__global__ __launch_bounds__(kBlock) void k_load_system(Layout L, const double* coef_nat, const double* b_nat,
                                                         const double* u, double* ured0, double* ured1,
                                                         double* ublack, double* coef, double* part_a,
                                                         double* part_b, Ctrl* C)
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
        const int64_t ci = ctile(L, colour, irow, m);
        double D = 1.0, s = b_nat[qi];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const double cm = coef_nat[qi * 8 + 2 * d], cp = coef_nat[qi * 8 + 2 * d + 1];
            coef[ci + (2 * d) * kTileSlots] = cm;
            coef[ci + (2 * d + 1) * kTileSlots] = cp;
            D += cm;
            D += cp;
            if (idx[d] > 1) s += cm * u[p - sd[d]];
            if (idx[d] < nn[d]) s += cp * u[p + sd[d]];
        }
        coef[ci + 8 * kTileSlots] = b_nat[qi];
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
    const double* coef;   // tiled coefficient + rhs block (both colours)
    double omega;
    double* part;         // this kernel's per-block partials
    const double* part_other;  // black partials of iterate k-1 (red check)
    Ctrl* C;
    int k;                // iteration number
    int check;            // red: test the stopping rule for iterate k-1
};

// Streaming accesses for data a sweep touches once (coefficients, rhs, own
// colour): non-temporal, so the neighbour rows of the other colour, which
// several blocks read, keep their place in L2.  Compile-time switch kept for
// measurement: SS4_STREAMING=0 gives plain accesses.
#ifndef SS4_STREAMING
#define SS4_STREAMING 1
#endif
__device__ __forceinline__ double ld_stream(const double* p)
{
#if SS4_STREAMING
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}
__device__ __forceinline__ void st_stream(double* p, double v)
{
#if SS4_STREAMING
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

typedef double dvec2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ dvec2 ld2(const double* p) { return *reinterpret_cast<const dvec2*>(p); }

__device__ __forceinline__ dvec2 ld2_stream(const double* p)
{
#if SS4_STREAMING
    return __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(p));
#else
    return *reinterpret_cast<const dvec2*>(p);
#endif
}

__device__ __forceinline__ void st2_stream(double* p, dvec2 v)
{
#if SS4_STREAMING
    __builtin_nontemporal_store(v, reinterpret_cast<dvec2*>(p));
#else
    *reinterpret_cast<dvec2*>(p) = v;
#endif
}

// End of a half-sweep: per-block partial of the squared residual rows; for a
// checking red sweep the last block adds the black partials of the same
// iterate and applies the stopping rule to iterate k-1.
template <int COLOR>
__device__ __forceinline__ void finish_sweep(const SweepArgs& a, double acc, double* lds, int* flag)
{
    Ctrl* C = a.C;
    const double bs = block_sum(acc, lds);
    if (threadIdx.x == 0) a.part[blockIdx.x] = bs;
    if (COLOR == 1 || !a.check) return;
    if (!arrive_last(&C->arrive[1], gridDim.x, flag)) return;
    const double Rr = sum_partials(a.part, gridDim.x, lds);
    const double Rb = sum_partials(a.part_other, gridDim.x, lds);
    if (threadIdx.x == 0) {
        const int kk = a.k - 1;
        const double R2 = Rb + Rr;
        const double R = sqrt(R2);
        C->rel_res = C->bn > 0.0 ? R / C->bn : R;
        bool stop = true;
        if (!(R2 < INFINITY)) C->status = SUBSURF4D_ENONFINITE;
        else if (R <= C->tol * C->bn) C->status = SUBSURF4D_OK;
        else if (kk >= C->max_iter) C->status = SUBSURF4D_NOT_CONVERGED;
        else stop = false;
        if (stop) {
            C->done = 1;
            C->iterations = kk;
            C->final_red = kk & 1;
        }
        C->arrive[1] = 0;
    }
}

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
        const double* cf = a.coef + ctile(L, COLOR, r, m);
        const double c0 = ld_stream(cf), c1 = ld_stream(cf + kTileSlots), c2 = ld_stream(cf + 2 * kTileSlots);
        const double c3 = ld_stream(cf + 3 * kTileSlots), c4 = ld_stream(cf + 4 * kTileSlots);
        const double c5 = ld_stream(cf + 5 * kTileSlots), c6 = ld_stream(cf + 6 * kTileSlots);
        const double c7 = ld_stream(cf + 7 * kTileSlots);
        const double* uo = a.uoth;
        double s = ld_stream(cf + 8 * kTileSlots);
        s += c0 * uo[ui - par] + c1 * uo[ui + 1 - par];
        s += c2 * uo[ui - sy] + c3 * uo[ui + sy];
        s += c4 * uo[ui - sz] + c5 * uo[ui + sz];
        s += c6 * uo[ui - st] + c7 * uo[ui + st];
        const double D = ((((((((1.0 + c0) + c1) + c2) + c3) + c4) + c5) + c6) + c7);
        const double ub = s / D;
        const double uold = ld_stream(a.uin + ui);
        st_stream(a.uout + ui, om * ub + om1 * uold);
        const double rres = COLOR == 0 ? D * (ub - uold) : D * om1 * (ub - uold);
        acc += rres * rres;
    }
    finish_sweep<COLOR>(a, acc, lds, &flag);
}

// Half-sweep in "t-marching" form.  A block owns a column tile (64 slots x 4
// y-rows at one z) and walks through the frames l = 1..N4.  Each thread keeps
// the other colour's values of its slot at l-1, l, l+1 in registers: they are
// its t-neighbours and one of its x-neighbours; the other x-neighbour comes
// from the adjacent lane.  y and z neighbours are read through the caches.
// Column tiles are dealt slot-tile fastest, then k, to the blocks of each XCD:
// the blocks resident together cover whole rows (the row-edge neighbours of
// lanes 0 and 63 and both halves of each coefficient tile are read at the same
// time) and adjacent planes (shared z neighbours in L2).  Same arithmetic as
// k_sweep (the red-black iterate does not depend on the visiting order).
template <int COLOR>
__global__ __launch_bounds__(kBlock) void k_sweep_tm(SweepArgs a)
{
    __shared__ double lds[4];
    __shared__ int flag;
    Ctrl* C = a.C;
    if (C->done) return;
    const Layout& L = a.L;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int ntm = (L.half + 63) >> 6;
    const int njb = (L.n2 + 3) >> 2;
    const int64_t ncol = (int64_t)ntm * njb * L.n3;
    const int64_t sy = L.rs, sz = (int64_t)L.p2 * L.rs, st = (int64_t)L.p2 * L.p3 * L.rs;
    const int64_t cst = (int64_t)L.n2 * L.n3 * L.ntm * kTileVals;   // coefficient stride between frames
    const int last_slot = L.n1 >> 1;                     // highest slot holding data in a row
    const double om = a.omega, om1 = 1.0 - a.omega;
    const double* __restrict__ uo = a.uoth;
    double acc = 0.0;
    for (TileWalk tw(ncol); tw.t < tw.end; tw.t += tw.step) {
        const int mt = (int)(tw.t % ntm);
        const int64_t t2 = tw.t / ntm;
        const int k = (int)(t2 % L.n3) + 1;
        const int jb = (int)(t2 / L.n3);
        const int j = jb * 4 + ty + 1;
        const int m = mt * 64 + tx;
        const bool jok = j <= L.n2;                      // uniform across the wave
        const bool sok = jok && m <= last_slot;
        const int64_t ub = ((int64_t)k * L.p2 + j) * L.rs + L.xoff + m;      // row (j,k,l=0)
        const int64_t cb = ctile(L, COLOR, ((int64_t)(k - 1) * L.n2 + (j - 1)), m);  // row (j,k,l=1)
        double Bm = sok ? uo[ub] : 0.0;
        double Bc = sok ? uo[ub + st] : 0.0;
        for (int l = 1; l <= L.n4; ++l) {
            const int64_t ui = ub + (int64_t)l * st;
            const double Bp = sok ? uo[ui + st] : 0.0;
            const int par = (COLOR + j + k + l) & 1;
            double left = __shfl_up(Bc, 1);
            double right = __shfl_down(Bc, 1);
            if (jok) {
                if (tx == 0 && par) left = uo[ui - 1];
                if (tx == 63 && !par && m + 1 <= last_slot) right = uo[ui + 1];
                const int cnt = par ? (L.n1 + 1) >> 1 : L.n1 >> 1;
                if (m < cnt) {
                    const double* cf = a.coef + cb + (int64_t)(l - 1) * cst;
                    const double c0 = ld_stream(cf), c1 = ld_stream(cf + kTileSlots);
                    const double c2 = ld_stream(cf + 2 * kTileSlots), c3 = ld_stream(cf + 3 * kTileSlots);
                    const double c4 = ld_stream(cf + 4 * kTileSlots), c5 = ld_stream(cf + 5 * kTileSlots);
                    const double c6 = ld_stream(cf + 6 * kTileSlots), c7 = ld_stream(cf + 7 * kTileSlots);
                    const double xl = par ? left : Bc;
                    const double xr = par ? Bc : right;
                    double s = ld_stream(cf + 8 * kTileSlots);
                    s += c0 * xl + c1 * xr;
                    s += c2 * uo[ui - sy] + c3 * uo[ui + sy];
                    s += c4 * uo[ui - sz] + c5 * uo[ui + sz];
                    s += c6 * Bm + c7 * Bp;
                    const double D = ((((((((1.0 + c0) + c1) + c2) + c3) + c4) + c5) + c6) + c7);
                    const double ubar = s / D;
                    const double uold = ld_stream(a.uin + ui);
                    st_stream(a.uout + ui, om * ubar + om1 * uold);
                    const double rres = COLOR == 0 ? D * (ubar - uold) : D * om1 * (ubar - uold);
                    acc += rres * rres;
                }
            }
            Bm = Bc;
            Bc = Bp;
        }
    }
    finish_sweep<COLOR>(a, acc, lds, &flag);
}

// Half-sweep, frame-marching with two cells per lane (rows of >= 64 slots,
// whose u rows are 128-byte aligned): a wave covers one 128-slot coefficient
// tile of one row, lane t owns slots m = 2t, 2t+1, and every stream moves 16
// bytes per lane.  A block walks column tiles (128 slots x 4 y-rows at one z),
// marching over the frames of each; tiles are dealt as for k_sweep_tm.
template <int COLOR>
__global__ __launch_bounds__(kBlock) void k_sweep_t2(SweepArgs a)
{
    __shared__ double lds[4];
    __shared__ int flag;
    Ctrl* C = a.C;
    if (C->done) return;
    const Layout& L = a.L;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int njb = (L.n2 + 3) >> 2;
    const int64_t ncol = (int64_t)L.ntm * njb * L.n3;
    const int64_t sy = L.rs, sz = (int64_t)L.p2 * L.rs, st = (int64_t)L.p2 * L.p3 * L.rs;
    const int64_t cst = (int64_t)L.n2 * L.n3 * L.ntm * kTileVals;
    const int last_slot = L.n1 >> 1;
    const double om = a.omega, om1 = 1.0 - a.omega;
    const double* __restrict__ uo = a.uoth;
    double acc = 0.0;
    for (TileWalk tw(ncol); tw.t < tw.end; tw.t += tw.step) {
        const int mt = (int)(tw.t % L.ntm);              // slot-tile fastest, then k (as k_sweep_tm)
        const int64_t t2 = tw.t / L.ntm;
        const int k = (int)(t2 % L.n3) + 1;
        const int jb = (int)(t2 / L.n3);
        const int j = jb * 4 + ty + 1;
        const int m = mt * kTileSlots + 2 * tx;
        const bool jok = j <= L.n2;                      // uniform across the wave
        const bool sok = jok && m <= last_slot;
        const int64_t ub = ((int64_t)k * L.p2 + j) * L.rs + L.xoff + m;
        const int64_t cb = ctile(L, COLOR, ((int64_t)(k - 1) * L.n2 + (j - 1)), m);
        const dvec2 zero2 = {0.0, 0.0};
        dvec2 Bm = sok ? ld2(uo + ub) : zero2;
        dvec2 Bc = sok ? ld2(uo + ub + st) : zero2;
        for (int l = 1; l <= L.n4; ++l) {
            const int64_t ui = ub + (int64_t)l * st;
            const dvec2 Bp = sok ? ld2(uo + ui + st) : zero2;
            const int par = (COLOR + j + k + l) & 1;
            double left = __shfl_up(Bc.y, 1);
            double right = __shfl_down(Bc.x, 1);
            if (jok) {
                if (tx == 0 && par) left = uo[ui - 1];
                if (tx == 63 && !par && m + 2 <= last_slot) right = uo[ui + 2];
                const int cnt = par ? (L.n1 + 1) >> 1 : L.n1 >> 1;
                if (m < cnt) {
                    const bool a1 = m + 1 < cnt;
                    const double* cf = a.coef + cb + (int64_t)(l - 1) * cst;
                    const dvec2 c0 = ld2_stream(cf), c1 = ld2_stream(cf + kTileSlots);
                    const dvec2 c2 = ld2_stream(cf + 2 * kTileSlots), c3 = ld2_stream(cf + 3 * kTileSlots);
                    const dvec2 c4 = ld2_stream(cf + 4 * kTileSlots), c5 = ld2_stream(cf + 5 * kTileSlots);
                    const dvec2 c6 = ld2_stream(cf + 6 * kTileSlots), c7 = ld2_stream(cf + 7 * kTileSlots);
                    const dvec2 bb = ld2_stream(cf + 8 * kTileSlots);
                    const dvec2 ym = ld2(uo + ui - sy), yp = ld2(uo + ui + sy);
                    const dvec2 zm = ld2(uo + ui - sz), zp = ld2(uo + ui + sz);
                    const dvec2 uold = ld2_stream(a.uin + ui);
                    // cell m: x-neighbours (m-par, m+1-par); cell m+1: (m+1-par, m+2-par)
                    const double xl0 = par ? left : Bc.x, xr0 = par ? Bc.x : Bc.y;
                    const double xl1 = par ? Bc.x : Bc.y, xr1 = par ? Bc.y : right;
                    double s0 = bb.x, s1 = bb.y;
                    s0 += c0.x * xl0 + c1.x * xr0;
                    s1 += c0.y * xl1 + c1.y * xr1;
                    s0 += c2.x * ym.x + c3.x * yp.x;
                    s1 += c2.y * ym.y + c3.y * yp.y;
                    s0 += c4.x * zm.x + c5.x * zp.x;
                    s1 += c4.y * zm.y + c5.y * zp.y;
                    s0 += c6.x * Bm.x + c7.x * Bp.x;
                    s1 += c6.y * Bm.y + c7.y * Bp.y;
                    const double D0 = ((((((((1.0 + c0.x) + c1.x) + c2.x) + c3.x) + c4.x) + c5.x) + c6.x) + c7.x);
                    const double D1 = ((((((((1.0 + c0.y) + c1.y) + c2.y) + c3.y) + c4.y) + c5.y) + c6.y) + c7.y);
                    const double ub0 = s0 / D0, ub1 = s1 / D1;
                    const double n0 = om * ub0 + om1 * uold.x;
                    const double n1 = om * ub1 + om1 * uold.y;
                    if (a1) {
                        const dvec2 nv = {n0, n1};
                        st2_stream(a.uout + ui, nv);
                    } else {
                        st_stream(a.uout + ui, n0);
                    }
                    const double r0 = COLOR == 0 ? D0 * (ub0 - uold.x) : D0 * om1 * (ub0 - uold.x);
                    const double r1 = COLOR == 0 ? D1 * (ub1 - uold.y) : D1 * om1 * (ub1 - uold.y);
                    acc += r0 * r0;
                    if (a1) acc += r1 * r1;
                }
            }
            Bm = Bc;
            Bc = Bp;
        }
    }
    finish_sweep<COLOR>(a, acc, lds, &flag);
}

// Plain 16-byte copy (bandwidth probe and counter calibration).
__global__ __launch_bounds__(kBlock) void k_copy_probe(const double2* __restrict__ src, double2* __restrict__ dst,
                                                       int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        dst[q] = src[q];
}

// Read-dominated probe: dst = sum of `reads` source chunks of n 16-byte
// elements each (reads streams in, one out, as the sweeps' traffic mix).
__global__ __launch_bounds__(kBlock) void k_stream_probe(const double2* __restrict__ src, double2* __restrict__ dst,
                                                         int64_t n, int reads)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        double2 acc = src[q];
        for (int r = 1; r < reads; ++r) {
            const double2 v = src[(int64_t)r * n + q];
            acc.x += v.x;
            acc.y += v.y;
        }
        dst[q] = acc;
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

// ghost layer of ub -> ghost layer of u
__global__ __launch_bounds__(kBlock) void k_copy_ghosts(Layout L, const double* __restrict__ ub, double* u)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < L.npad; p += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(p % L.p1);
        const int64_t prow = p / L.p1;
        const int j = (int)(prow % L.p2);
        const int64_t t2 = prow / L.p2;
        const int k = (int)(t2 % L.p3);
        const int l = (int)(t2 / L.p3);
        const bool inside = i >= 1 && i <= L.n1 && j >= 1 && j <= L.n2 && k >= 1 && k <= L.n3 && l >= 1 && l <= L.n4;
        if (!inside) u[p] = ub[p];
    }
}

// Outcome of the solve into a device-accessible result (enqueue-only calls).
__global__ void k_write_result(const Ctrl* C, subsurf4d_result* res, int sweeps_per_pass)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        res->status = C->status;
        res->iterations = sweeps_per_pass > 0 ? C->outer * sweeps_per_pass : C->iterations;
        res->outer_iterations = C->outer;
        res->reserved = 0;
        res->rel_residual = C->rel_res;
        res->bnorm = C->bn;
    }
}

int sweep_grid(const Layout& L, int variant)
{
    int64_t work;
    int res;
    if (variant == 2) {
        work = (int64_t)L.ntm * ((L.n2 + 3) >> 2) * L.n3;
        res = resident_grid(reinterpret_cast<const void*>(&k_sweep_t2<0>)) / 2;
        const int64_t g = work < res ? work : res;
        return (int)((g + kXcd - 1) / kXcd * kXcd);
    }
    if (variant == 1) {
        // half the resident size: fewer streams in flight per XCD keep DRAM
        // pages and the shared neighbour rows better (measured on the
        // 512x512x96x16 volume: 4.22 ms vs 4.25 ms per half-sweep)
        work = (int64_t)L.ntm * ((L.n2 + 3) >> 2) * L.n3;
        res = resident_grid(reinterpret_cast<const void*>(&k_sweep_tm<0>)) / 2;
    } else {
        work = (int64_t)L.ntm * ((L.nrow_int + 3) >> 2);
        res = resident_grid(reinterpret_cast<const void*>(&k_sweep<0>));
    }
    const int64_t g = work < res ? work : res;
    return (int)((g + kXcd - 1) / kXcd * kXcd);
}

// Sweep kernel choice.  2 (default for rows of >= 64 slots): frame-marching
// with two cells per lane and 16-byte accesses (k_sweep_t2), the fastest
// measured on the 512x512x96x16 volume (3.95 ms vs 4.22 ms per half-sweep);
// 1 (default for narrower rows): frame-marching, one cell per lane
// (k_sweep_tm); 0: row tiles (k_sweep).  SUBSURF4D_SWEEP=r|t|p selects one
// explicitly (all three give the same iterates).
int sweep_variant(const Layout& L)
{
    const bool wide = L.half >= 64;   // 128-byte aligned u rows, pairs stay in the row
    static const char* env = getenv("SUBSURF4D_SWEEP");
    if (env && env[0] == 'r') return 0;
    if (env && env[0] == 't') return 1;
    return wide ? 2 : 1;
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
    double* pa = ws_ptr<double>(ws, P.part_a);
    double* pb = ws_ptr<double>(ws, P.part_b);
    double tol;
    int max_iter;
    effective_stop(sp, &tol, &max_iter);
    const int check_every = sp.check_every > 0 ? sp.check_every : 1;
    const int variant = sweep_variant(L);
    const int grid = sweep_grid(L, variant);

    SweepArgs red{}, black{};
    red.L = black.L = L;
    red.omega = black.omega = sp.omega;
    red.C = black.C = C;
    red.coef = coef;
    black.coef = coef;
    red.part = pa;
    red.part_other = pb;
    black.part = pb;
    black.uin = black.uout = ublack;
    red.uoth = ublack;

    // red half-sweep k (which also tests iterate k-1) and black half-sweep k;
    // every launch returns at once after the stopping rule has been met
    auto enqueue_iteration = [&](int k) {
        red.k = k;
        red.uin = ured[(k - 1) & 1];
        red.uout = ured[k & 1];
        red.check = (k >= 2) && (((k - 1) % check_every == 0) || (k - 1 >= max_iter));
        if (variant == 2) k_sweep_t2<0><<<grid, kBlock, 0, s>>>(red);
        else if (variant == 1) k_sweep_tm<0><<<grid, kBlock, 0, s>>>(red);
        else k_sweep<0><<<grid, kBlock, 0, s>>>(red);
        if (k <= max_iter) {
            black.k = k;
            black.uoth = ured[k & 1];
            if (variant == 2) k_sweep_t2<1><<<grid, kBlock, 0, s>>>(black);
            else if (variant == 1) k_sweep_tm<1><<<grid, kBlock, 0, s>>>(black);
            else k_sweep<1><<<grid, kBlock, 0, s>>>(black);
        }
    };
    if (sp.flags & SUBSURF4D_FLAG_ASYNC) {
        // enqueue-only: every iteration up to the cap, no host read
        for (int k = 1; k <= max_iter + 1; ++k) enqueue_iteration(k);
        SS4_LAUNCHED("sweeps");
        return 0;
    }

    Ctrl hc;
    SS4_HIP(hipMemcpyAsync(&hc, C, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    SS4_HIP(hipStreamSynchronize(s));
    SweepTimer timer(s);
    int k = 1;
    int chunk = sp.iter_hint > 0 ? sp.iter_hint + 1 : 8;
    while (!hc.done) {
        timer.begin();
        for (int c = 0; c < chunk && k <= max_iter + 1; ++c, ++k) enqueue_iteration(k);
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

int run_copy_probe(const void* src, void* dst, size_t bytes, int reps, double* ms, hipStream_t s)
{
    const int64_t n = (int64_t)(bytes / 16);
    hipEvent_t a, b;
    SS4_HIP(hipEventCreate(&a));
    SS4_HIP(hipEventCreate(&b));
    const int grid = 8192;
    k_copy_probe<<<grid, kBlock, 0, s>>>(static_cast<const double2*>(src), static_cast<double2*>(dst), n);
    SS4_HIP(hipEventRecord(a, s));
    for (int r = 0; r < reps; ++r)
        k_copy_probe<<<grid, kBlock, 0, s>>>(static_cast<const double2*>(src), static_cast<double2*>(dst), n);
    SS4_HIP(hipEventRecord(b, s));
    SS4_HIP(hipEventSynchronize(b));
    float t = 0.f;
    SS4_HIP(hipEventElapsedTime(&t, a, b));
    *ms = (double)t / reps;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    SS4_LAUNCHED("copy probe");
    return 0;
}

int run_stream_probe(const void* src, void* dst, size_t bytes, int reads, int reps, double* ms, hipStream_t s)
{
    const int64_t n = (int64_t)(bytes / 16);
    hipEvent_t a, b;
    SS4_HIP(hipEventCreate(&a));
    SS4_HIP(hipEventCreate(&b));
    const int grid = 8192;
    const double2* sp = static_cast<const double2*>(src);
    double2* dp = static_cast<double2*>(dst);
    k_stream_probe<<<grid, kBlock, 0, s>>>(sp, dp, n, reads);
    SS4_HIP(hipEventRecord(a, s));
    for (int r = 0; r < reps; ++r) k_stream_probe<<<grid, kBlock, 0, s>>>(sp, dp, n, reads);
    SS4_HIP(hipEventRecord(b, s));
    SS4_HIP(hipEventSynchronize(b));
    float t = 0.f;
    SS4_HIP(hipEventElapsedTime(&t, a, b));
    *ms = (double)t / reps;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    SS4_LAUNCHED("stream probe");
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
    a.ub = u;
    a.coef_nat = coef;
    a.b_nat = b;
    k_assemble<kNatural><<<grid_for(L.npad), kBlock, 0, s>>>(a);
    SS4_LAUNCHED("assemble (export)");
    return 0;
}

int launch_assembly(const WsPlan& P, double h, const double* G, const double* w, const double* ub,
                    const subsurf4d_step_params& sp, void* coef16, void* ws, hipStream_t s)
{
    AsmArgs a{};
    a.L = P.L;
    a.th2 = sp.tau / (h * h);
    a.eps2 = sp.eps * sp.eps;
    a.inv_h = 1.0 / h;
    a.G = G;
    a.w = w;
    a.ub = ub ? ub : w;
    a.ured0 = ws_ptr<double>(ws, P.ured0);
    a.ured1 = ws_ptr<double>(ws, P.ured1);
    a.ublack = ws_ptr<double>(ws, P.ublack);
    a.coef = ws_ptr<double>(ws, P.coef);
    a.coef16 = static_cast<uint4*>(coef16);
    a.part_a = ws_ptr<double>(ws, P.part_a);
    a.part_b = ws_ptr<double>(ws, P.part_b);
    a.C = ws_ptr<Ctrl>(ws, P.ctrl);
    const Layout& L = P.L;
    k_ghost_split<<<grid_for(L.nrow_pad * 64), kBlock, 0, s>>>(L, a.ub, a.ured0, a.ured1, a.ublack);
    const int64_t ncol = (int64_t)((L.n1 + 63) >> 6) * ((L.n2 + 3) >> 2) * L.n3;
    // SUBSURF4D_ASM_PREFETCH=0|1 selects the slab loading: loads of the next
    // frame issued after the barrier and kept in flight during the cell
    // arithmetic (1), or issued just before the frame's LDS store (0); both
    // give the same bits
    static const char* env = getenv("SUBSURF4D_ASM_PREFETCH");
    const bool prefetch = !(env && env[0] == '0');
    const void* kern = prefetch ? reinterpret_cast<const void*>(&k_assemble_cols<true>)
                                : reinterpret_cast<const void*>(&k_assemble_cols<false>);
    const int res = resident_grid(kern);
    const int64_t g = ncol < res ? ncol : res;
    const int grid = (int)((g + kXcd - 1) / kXcd * kXcd);
    if (prefetch) k_assemble_cols<true><<<grid, kBlock, 0, s>>>(a);
    else k_assemble_cols<false><<<grid, kBlock, 0, s>>>(a);
    SS4_LAUNCHED("assemble");
    return 0;
}

int run_step(const WsPlan& P, double h, const double* G, const double* ub, const subsurf4d_centre* centres,
             int nc, const int32_t* owner, double* u, const subsurf4d_step_params& sp, subsurf4d_result* res,
             void* ws, hipStream_t s)
{
    const Layout& L = P.L;
    Ctrl* C = ws_ptr<Ctrl>(ws, P.ctrl);
    int rc;
    if (sp.precision == SUBSURF4D_MIXED) {
        rc = run_mixed_solve(P, h, G, u, ub, sp, res, ws, s);
        if (rc < 0) return rc;
        rc = run_unsplit(P, u, ws, s);
        if (rc < 0) return rc;
    } else {
        double tol;
        int max_iter;
        effective_stop(sp, &tol, &max_iter);
        k_ctrl_init<<<1, 64, 0, s>>>(C, tol, max_iter);
        rc = launch_assembly(P, h, G, u, ub, sp, nullptr, ws, s);
        if (rc < 0) return rc;
        rc = run_sor_loop(P, sp, ws, s, res);
        if (rc < 0) return rc;
        rc = run_unsplit(P, u, ws, s);
        if (rc < 0) return rc;
    }
    if (ub && ub != u) {
        // the new level carries its Dirichlet data in its ghost layer
        k_copy_ghosts<<<grid_for(L.npad), kBlock, 0, s>>>(L, ub, u);
        SS4_LAUNCHED("ghost layer");
    }
    if (sp.rescale && nc > 0) {
        const int r2 = run_rescale(P, centres, nc, sp.ball_r, owner, u, ws, s);
        if (r2 < 0) return r2;
    }
    if (sp.flags & SUBSURF4D_FLAG_ASYNC) {
        if (res) {
            k_write_result<<<1, 64, 0, s>>>(C, res, sp.precision == SUBSURF4D_MIXED ? sp.inner_sweeps : 0);
            SS4_LAUNCHED("result");
        }
        return 0;
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
                                                      ws_ptr<double>(ws, P.coef), ws_ptr<double>(ws, P.part_a),
                                                      ws_ptr<double>(ws, P.part_b), C);
    SS4_LAUNCHED("load system");
    int rc = run_sor_loop(P, sp, ws, s, res);
    if (rc < 0) return rc;
    rc = run_unsplit(P, u, ws, s);
    if (rc < 0) return rc;
    if (sp.flags & SUBSURF4D_FLAG_ASYNC) {
        if (res) {
            k_write_result<<<1, 64, 0, s>>>(C, res, 0);
            SS4_LAUNCHED("result");
        }
        return 0;
    }
    SS4_HIP(hipStreamSynchronize(s));
    return res ? res->status : 0;
}

}  // namespace ss4
