// Time-step kernels: assembly of the finite-volume system from
// reduced-diamond-cell face gradients (Sec. 3.2.2, the uniform-h system with
// A_eps and A_eps-bar), red-black SOR half-sweeps with the residual norm fused
// in, and the host driver of the iteration.
#include <cmath>
#include <cstdlib>

#include "ss4_internal.hpp"
#include "ss4_sweep.hpp"

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
// Store of an assembly output: non-temporal (NTS) for the column kernel, so
// that the ~90 B per cell written do not push the neighbour planes of w and G
// that the adjacent blocks are about to read out of L2.
template <bool NTS, typename T>
__device__ __forceinline__ void put(T* p, T v)
{
    if (NTS) __builtin_nontemporal_store(v, p);
    else *p = v;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// The t-face carried from frame to frame by a thread that marches the frames:
// the -t face of its cell at frame l is the +t face of its cell at frame l-1,
// whose q and 1/sqrt(eps^2 + q) were formed from the same values in the same
// order one frame earlier.
struct TFace {
    double q = 0.0, rs = 0.0;
    bool valid = false;
};

template <int MODE, bool NTS, typename WAt, typename GAt>
__device__ __forceinline__ void assemble_cell(const AsmArgs& a, int64_t p, int i, int j, int k, int l, int colour,
                                              int m, WAt&& wat, GAt&& gat, double& acc_b, double& acc_r,
                                              TFace* tf = nullptr)
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
    const bool carried = tf && tf->valid;            // -t face known from the previous frame
    double q[8];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const bool skip_m = d == 3 && carried;
        const double gnm = (w0 - wm[d]) * a.inv_h;   // normal, -e_d face
        const double gnp = (wp[d] - w0) * a.inv_h;   // normal, +e_d face
        double qm = gnm * gnm, qp = gnp * gnp;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t == d) continue;
            const double wpt = wp[t], wmt = wm[t];
            const double dp_pt = w2(d, 1, t, 1), dp_mt = w2(d, 1, t, -1);
            const double tp = ((wpt + dp_pt) - (wmt + dp_mt)) * (0.25 * a.inv_h);
            qp += tp * tp;
            if (!skip_m) {
                const double dm_pt = w2(d, -1, t, 1), dm_mt = w2(d, -1, t, -1);
                const double tm = ((dm_pt + wpt) - (dm_mt + wmt)) * (0.25 * a.inv_h);
                qm += tm * tm;
            }
        }
        q[2 * d] = skip_m ? tf->q : qm;
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
        // G/A as a product with the reciprocal square root (a few ulps from
        // the quotient by the rounded root, at a third of the instructions;
        // the batched assembly forms it the same way)
        const double rm = (d == 3 && carried) ? tf->rs : rsqrt(a.eps2 + q[2 * d]);
        const double rp = rsqrt(a.eps2 + q[2 * d + 1]);
        c[2 * d] = scale * gm * rm;
        c[2 * d + 1] = scale * gp * rp;
        if (d == 3 && tf) {
            tf->q = q[7];
            tf->rs = rp;
            tf->valid = true;
        }
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
        for (int f = 0; f < 8; ++f) put<NTS>(a.coef + ci + f * kTileSlots, c[f]);
        put<NTS>(a.coef + ci + 8 * kTileSlots, w0);
        if (a.coef16) {
            const double inv = 1.0 / D;
            uint32_t h[8];
#pragma unroll
            for (int f = 0; f < 8; ++f) h[f] = bf16_bits((float)(c[f] * inv));
            const u32x4 rec = {h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
            put<NTS>(reinterpret_cast<u32x4*>(a.coef16 + mrec(L, colour, irow, m)), rec);
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
        assemble_cell<MODE, false>(
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
// into a ring of four frame slots (one barrier per frame), so every w value
// comes from LDS and each frame's slab is read from memory once per block.  The t-face G of the frame
// below is kept in a register from the previous frame.  Tiles of one XCD are
// consecutive (x-tile fastest, then z), so the neighbour planes a block loads
// are loaded by the blocks beside it at about the same time (L2 hits).  Ghost
// cells are written by k_ghost_split.
constexpr int kAx = 66, kAy = 6, kAz = 3;                  // slab: x with halo, y rows with halo, z planes
constexpr int kSlab = kAx * kAy * kAz;                     // doubles per frame slot
constexpr int kRing = 4;                                   // frame slots: l-1, l, l+1 and the one being filled

template <bool PREFETCH, bool NTS>
__global__ __launch_bounds__(kBlock) void k_assemble_cols(AsmArgs a)
{
    __shared__ double lds[4];
    __shared__ int flag;
    __shared__ double slab[kRing][kSlab];
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
        // assembled, and then to the ring slot lf % kRing
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
        int64_t soff[kPer];              // this thread's slab entries, once per tile
#pragma unroll
        for (int r = 0; r < kPer; ++r) soff[r] = source(threadIdx.x + r * kBlock);
        auto fetch = [&](int lf) {
            const double* fw = a.w + (int64_t)lf * s4;
#pragma unroll
            for (int r = 0; r < kPer; ++r) pf[r] = soff[r] >= 0 ? fw[soff[r]] : 0.0;
        };
        auto store = [&](int lf) {
            double* dst = slab[lf % kRing];
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                const int q = threadIdx.x + r * kBlock;
                if (q < kSlab) dst[q] = pf[r];
            }
        };
        auto load = [&](int lf) {               // without prefetch: straight from memory to LDS
            double* dst = slab[lf % kRing];
            const double* fw = a.w + (int64_t)lf * s4;
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                const int q = threadIdx.x + r * kBlock;
                if (q < kSlab) dst[q] = soff[r] >= 0 ? fw[soff[r]] : 0.0;
            }
        };
        __syncthreads();                 // the previous tile's last frame is no longer read
        load(0);
        load(1);
        if (PREFETCH) fetch(2);
        double gt_below = active ? a.G[3 * L.npad + ((int64_t)k * L.p2 + j) * L.p1 + i] : 0.0;   // G_t of frame 0
        TFace tface;                     // the +t face of the previous frame's cell
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
                const double w0 = slab[l % kRing][(1 * kAy + ty + 1) * kAx + tx + 1];
                const int64_t us = prow * L.rs + L.xoff + m;
                // the red value goes to the first ping-pong buffer only: the
                // first red half-sweep writes every interior cell of the second
                // before anything reads it
                if (colour == 0) put<NTS>(a.ured0 + us, w0);
                else put<NTS>(a.ublack + us, w0);
                const double gt_here = a.G[3 * L.npad + p];
                const int sl[3] = {(l - 1) % kRing, l % kRing, (l + 1) % kRing};   // slots of frames l-1, l, l+1
                assemble_cell<kSplit, NTS>(
                    a, p, i, j, k, l, colour, m,
                    [&](int di, int dj, int dk, int dl) {
                        return slab[sl[dl + 1]][((dk + 1) * kAy + ty + 1 + dj) * kAx + tx + 1 + di];
                    },
                    [&](int d, int plus) {
                        if (d == 3) return plus ? gt_here : gt_below;
                        const int64_t o = d == 0 ? 1 : (d == 1 ? s2 : s3);
                        return a.G[(int64_t)d * L.npad + p - (plus ? 0 : o)];
                    },
                    acc_b, acc_r, &tface);
                gt_below = gt_here;
            }
            // no barrier here: the slot refilled next (frame l+2's) held frame
            // l-2, which every wave finished reading before the barrier above
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

// Plain 16-byte copy (bandwidth probe and counter calibration).
__global__ __launch_bounds__(kBlock) void k_copy_probe(const double2* __restrict__ src, double2* __restrict__ dst,
                                                       int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        dst[q] = src[q];
}

// Read-dominated probe over `reads` source chunks of n 16-byte elements.
// WRITE: dst = element-wise sum of the chunks (reads streams in, one out, as
// the sweeps' traffic mix); otherwise dst[block] = the block's share of the
// total (reads only).  Each thread keeps kProbeU non-temporal 16-byte loads
// per chunk in flight, which is what it takes to reach the chip's streaming
// rate.
constexpr int kProbeU = 4;

template <bool WRITE>
__global__ __launch_bounds__(kBlock) void k_stream_probe(const double2* __restrict__ src, double2* __restrict__ dst,
                                                         int64_t n, int reads)
{
    typedef double dv2 __attribute__((ext_vector_type(2)));
    const dv2* s = reinterpret_cast<const dv2*>(src);
    dv2* d = reinterpret_cast<dv2*>(dst);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    dv2 tot = {0.0, 0.0};
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; base < n; base += stride * kProbeU) {
        dv2 acc[kProbeU];
#pragma unroll
        for (int u = 0; u < kProbeU; ++u) acc[u] = dv2{0.0, 0.0};
#pragma unroll 2
        for (int r = 0; r < reads; ++r) {
            const dv2* sr = s + (int64_t)r * n;
#pragma unroll
            for (int u = 0; u < kProbeU; ++u) {
                const int64_t q = base + u * stride;
                if (q < n) acc[u] += __builtin_nontemporal_load(sr + q);
            }
        }
#pragma unroll
        for (int u = 0; u < kProbeU; ++u) {
            const int64_t q = base + u * stride;
            if (q >= n) continue;
            if (WRITE) __builtin_nontemporal_store(acc[u], d + q);
            else tot += acc[u];
        }
    }
    if (!WRITE) {
        __shared__ double lds[4];
        const double bx = block_sum(tot.x, lds);
        const double by = block_sum(tot.y, lds);
        if (threadIdx.x == 0) dst[blockIdx.x] = make_double2(bx, by);
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
        res = (int)((int64_t)resident_grid(reinterpret_cast<const void*>(&k_sweep_t2<0>)) * sweep_grid_percent(50) / 100);
        if (res > kGridCap) res = kGridCap;    // the per-block partial arrays hold kGridCap entries
        const int64_t g = work < res ? work : res;
        return (int)((g + kXcd - 1) / kXcd * kXcd);
    }
    if (variant == 5) {
        // 64 KB of LDS per block: two blocks per CU at the resident size, the
        // occupancy the immediate-store form has at half its resident grid
        work = (int64_t)L.ntm * ((L.n2 + 3) >> 2) * L.n3;
        res = (int)((int64_t)resident_grid(reinterpret_cast<const void*>(&k_sweep_t2<0, 4, 16>)) *
                    sweep_grid_percent(100) / 100);
        if (res > kGridCap) res = kGridCap;
        const int64_t g = work < res ? work : res;
        return (int)((g + kXcd - 1) / kXcd * kXcd);
    }
    if (variant == 7 || variant == 9) {
        // 128 KB of LDS per block: one block per CU at the resident size
        const int rows = variant == 9 ? 16 : 8;
        work = (int64_t)L.ntm * ((L.n2 + rows - 1) / rows) * L.n3;
        const void* kern = variant == 7 ? reinterpret_cast<const void*>(&k_sweep_t2<0, 8, 16>)
                                        : reinterpret_cast<const void*>(&k_sweep_t2<0, 16, 8>);
        res = (int)((int64_t)resident_grid_bs(kern, 64 * rows) * sweep_grid_percent(100) / 100);
        if (res > kGridCap) res = kGridCap;
        const int64_t g = work < res ? work : res;
        return (int)((g + kXcd - 1) / kXcd * kXcd);
    }
    if (variant == 3) {
        work = (int64_t)L.ntm * ((L.n2 + 7) >> 3) * L.n3;
        res = resident_grid_bs(reinterpret_cast<const void*>(&k_sweep_t2<0, 8>), 512) / 2;
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

// Sweep kernel choice.  9 (default for rows of >= 64 slots): frame-marching
// with two cells per lane and 16-byte accesses (k_sweep_t2) in 16-row blocks,
// new values held in LDS and written after a block barrier every 8 frames,
// the fastest measured on the 512x512x96x16 volume (3.566 ms per half-sweep;
// 3.603 with 8-row blocks and 16 frames (7), 3.785 with 4-row blocks and 16
// frames (5), 3.954 storing each frame at once (2), 4.22 with one cell per
// lane); 1 (default for narrower rows): frame-marching, one cell per lane
// (k_sweep_tm); 0: row tiles (k_sweep); 3: two cells per lane, 8-row blocks,
// storing at once.  SUBSURF4D_SWEEP=r|t|p|8|d|D selects one explicitly (all
// give the same iterates).
int sweep_variant(const Layout& L)
{
    const bool wide = L.half >= 64;   // 128-byte aligned u rows, pairs stay in the row
    const char* env = getenv("SUBSURF4D_SWEEP");     // read per solve, so a process can switch
    if (env && env[0] == 'r') return 0;
    if (env && env[0] == 't') return 1;
    // 3: the two-cell form with 8 y-rows per block (fewer neighbour rows
    // outside each column tile); SUBSURF4D_SWEEP=8 selects it
    if (env && env[0] == '8') return wide ? 3 : 1;
    // 2: the two-cell form storing each frame's new values at once (SUBSURF4D_SWEEP=p)
    if (env && env[0] == 'p') return wide ? 2 : 1;
    // 5: 4-row blocks with the deferred writes, 16 frames (SUBSURF4D_SWEEP=d);
    // 7: 8-row blocks, 16 frames (SUBSURF4D_SWEEP=D)
    if (env && env[0] == 'd') return wide ? 5 : 1;
    if (env && env[0] == 'D') return wide ? 7 : 1;
    // 9 (default for rows of >= 64 slots): the two-cell form in 16-row blocks
    // of 1024 threads, new values held in LDS (128 KB) and written after a
    // block barrier every 8 frames
    return wide ? 9 : 1;
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
        if (variant == 5) k_sweep_t2<0, 4, 16><<<grid, kBlock, 0, s>>>(red);
        else if (variant == 7) k_sweep_t2<0, 8, 16><<<grid, 512, 0, s>>>(red);
        else if (variant == 9) k_sweep_t2<0, 16, 8><<<grid, 1024, 0, s>>>(red);
        else if (variant == 3) k_sweep_t2<0, 8><<<grid, 512, 0, s>>>(red);
        else if (variant == 2) k_sweep_t2<0><<<grid, kBlock, 0, s>>>(red);
        else if (variant == 1) k_sweep_tm<0><<<grid, kBlock, 0, s>>>(red);
        else k_sweep<0><<<grid, kBlock, 0, s>>>(red);
        if (k <= max_iter) {
            black.k = k;
            black.uoth = ured[k & 1];
            if (variant == 5) k_sweep_t2<1, 4, 16><<<grid, kBlock, 0, s>>>(black);
            else if (variant == 7) k_sweep_t2<1, 8, 16><<<grid, 512, 0, s>>>(black);
            else if (variant == 9) k_sweep_t2<1, 16, 8><<<grid, 1024, 0, s>>>(black);
            else if (variant == 3) k_sweep_t2<1, 8><<<grid, 512, 0, s>>>(black);
            else if (variant == 2) k_sweep_t2<1><<<grid, kBlock, 0, s>>>(black);
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

int stream_probe_grid(size_t bytes)
{
    const int64_t n = (int64_t)(bytes / 16);
    const int64_t g = (n + (int64_t)kBlock * kProbeU - 1) / ((int64_t)kBlock * kProbeU);
    return (int)(g < 65536 ? g : 65536);
}

int run_stream_probe(const void* src, void* dst, size_t bytes, int reads, int writes, int reps, double* ms,
                     hipStream_t s)
{
    const int64_t n = (int64_t)(bytes / 16);
    hipEvent_t a, b;
    SS4_HIP(hipEventCreate(&a));
    SS4_HIP(hipEventCreate(&b));
    const int grid = stream_probe_grid(bytes);
    const double2* sp = static_cast<const double2*>(src);
    double2* dp = static_cast<double2*>(dst);
    auto launch = [&] {
        if (writes) k_stream_probe<true><<<grid, kBlock, 0, s>>>(sp, dp, n, reads);
        else k_stream_probe<false><<<grid, kBlock, 0, s>>>(sp, dp, n, reads);
    };
    launch();
    SS4_HIP(hipEventRecord(a, s));
    for (int r = 0; r < reps; ++r) launch();
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
    // SUBSURF4D_ASM_NT=0|1: plain or non-temporal stores of the outputs (same bits)
    const char* env = getenv("SUBSURF4D_ASM_PREFETCH");
    const char* env_nt = getenv("SUBSURF4D_ASM_NT");
    const bool prefetch = !(env && env[0] == '0');
    const bool nts = !(env_nt && env_nt[0] == '0');
    const void* kern = prefetch ? (nts ? reinterpret_cast<const void*>(&k_assemble_cols<true, true>)
                                       : reinterpret_cast<const void*>(&k_assemble_cols<true, false>))
                                : (nts ? reinterpret_cast<const void*>(&k_assemble_cols<false, true>)
                                       : reinterpret_cast<const void*>(&k_assemble_cols<false, false>));
    const int res = resident_grid(kern);
    const int64_t g = ncol < res ? ncol : res;
    const int grid = (int)((g + kXcd - 1) / kXcd * kXcd);
    if (prefetch && nts) k_assemble_cols<true, true><<<grid, kBlock, 0, s>>>(a);
    else if (prefetch) k_assemble_cols<true, false><<<grid, kBlock, 0, s>>>(a);
    else if (nts) k_assemble_cols<false, true><<<grid, kBlock, 0, s>>>(a);
    else k_assemble_cols<false, false><<<grid, kBlock, 0, s>>>(a);
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

// SUBSURF4D_SWEEP_GRID=<percent> sizes the grids of the frame-marching FP64
// and FP32 sweeps as that share of the resident grid (defaults: the caller's
// `dflt`); the tile walk gives the same iterate for any grid.
int sweep_grid_percent(int dflt)
{
    const char* env = getenv("SUBSURF4D_SWEEP_GRID");
    const int pc = env ? atoi(env) : dflt;
    return pc < 1 ? 1 : (pc > 400 ? 400 : pc);
}

}  // namespace ss4
