// Red-black SOR half-sweeps of the FP64 system with the stopping-rule
// residual fused in (Sec. 3.2.2, RED-BLACK paragraph): the hot loop of a time
// step.  Included by the step driver (ss4_solve.hip) only.
#pragma once

#include "ss4_internal.hpp"

namespace ss4 {
namespace {

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

// Sum over a block of NW waves in a fixed order (the 4-wave case is
// block_sum); valid in thread 0.
template <int NW>
__device__ __forceinline__ double block_sum_w(double v, double* lds)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        t = lds[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) t += lds[w];
    }
    __syncthreads();
    return t;
}

template <int NW>
__device__ __forceinline__ double sum_partials_w(const double* part, int n, double* lds)
{
    double s = 0.0;
    for (int q = threadIdx.x; q < n; q += 64 * NW) s += part[q];
    return block_sum_w<NW>(s, lds);
}

// End of a half-sweep: per-block partial of the squared residual rows; for a
// checking red sweep the last block adds the black partials of the same
// iterate and applies the stopping rule to iterate k-1.
template <int COLOR, int NW = 4>
__device__ __forceinline__ void finish_sweep(const SweepArgs& a, double acc, double* lds, int* flag)
{
    Ctrl* C = a.C;
    const double bs = block_sum_w<NW>(acc, lds);
    if (threadIdx.x == 0) a.part[blockIdx.x] = bs;
    if (COLOR == 1 || !a.check) return;
    if (!arrive_last(&C->arrive[1], gridDim.x, flag)) return;
    const double Rr = sum_partials_w<NW>(a.part, gridDim.x, lds);
    const double Rb = sum_partials_w<NW>(a.part_other, gridDim.x, lds);
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
// bytes per lane.  A block of NW waves walks column tiles (128 slots x NW
// y-rows at one z), marching over the frames of each; tiles are dealt as for
// k_sweep_tm.
// DF > 0: a thread's new values of up to DF frames wait in LDS and are
// written after a block barrier, so the block's waves write together: the
// write stream then interleaves less with the reads of the other blocks.
template <int COLOR, int NW = 4, int DF = 0>
__global__ __launch_bounds__(64 * NW) void k_sweep_t2(SweepArgs a)
{
    constexpr bool DEFER = DF > 0;
    constexpr int kDeferFrames = DEFER ? DF : 1;
    __shared__ double lds[NW];
    __shared__ int flag;
    __shared__ dvec2 obuf[kDeferFrames][DEFER ? 64 * NW : 1];
    Ctrl* C = a.C;
    if (C->done) return;
    const Layout& L = a.L;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int njb = (L.n2 + NW - 1) / NW;
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
        const int j = jb * NW + ty + 1;
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
                    if (DEFER) {
                        const dvec2 nv = {n0, n1};
                        obuf[(l - 1) % kDeferFrames][threadIdx.x] = nv;
                    } else if (a1) {
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
            if (DEFER && (l % kDeferFrames == 0 || l == L.n4)) {
                // the same l and N4 in every wave: a uniform barrier
                __syncthreads();
                if (jok) {
                    const int l0 = (l - 1) / kDeferFrames * kDeferFrames + 1;
                    for (int lf = l0; lf <= l; ++lf) {
                        const int parf = (COLOR + j + k + lf) & 1;
                        const int cntf = parf ? (L.n1 + 1) >> 1 : L.n1 >> 1;
                        if (m >= cntf) continue;
                        const dvec2 nv = obuf[(lf - 1) % kDeferFrames][threadIdx.x];
                        double* dst = a.uout + ub + (int64_t)lf * st;
                        if (m + 1 < cntf) st2_stream(dst, nv);
                        else st_stream(dst, nv.x);
                    }
                }
            }
        }
    }
    finish_sweep<COLOR, NW>(a, acc, lds, &flag);
}

}  // namespace
}  // namespace ss4
