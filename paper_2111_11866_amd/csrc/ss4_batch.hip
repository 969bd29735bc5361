// Batched time step over many independent windows (one job per window), in
// mixed precision: FP32 red-black sweeps on BF16 scaled coefficients inside
// an FP64 iterative refinement (as ss4_mixed.hip), for every job at once.
//
// Layout per job ("flat"): for each colour, the cells of interior row r and
// slot m = (i-1)>>1 are numbered q = r*half + m (half = ceil(N1/2)); a slot is
// a cell of that colour when m < ceil/floor(N1/2) for the row's parity.  The
// colour-split iterate x (FP64) and correction d (FP32) keep every padded row
// with row stride half+2 (slot m at 1+m, ghosts at 0 and N1>>1 + 1).
// Coefficients are tiled by 128 consecutive q (9 FP64 fields per tile), the
// BF16 records and r/D are dense in q.  Small windows waste no lanes on row
// padding: 256 consecutive q of one colour form a work item.
//
// Every launch walks a global list of work items with a resident-size grid,
// each XCD a contiguous chunk of it in rounds.  The refinement kernels walk a list
// compacted to the unfinished jobs after every stopping decision, so the
// remaining work of the slow jobs is spread over the whole device.  Each job
// reduces its own per-item partial sums in a fixed order in a kernel of its
// own, so a job's result does not depend on which other jobs share the launch
// or on which block visits which item.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "ss4_batch.hpp"

namespace ss4 {

namespace {
__global__ void kb_init(BTable T, double tol, int max_outer)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < T.n_jobs; j += gridDim.x * blockDim.x) {
        Ctrl* C = T.jobs[j].C;
        for (int a = 0; a < 4; ++a) C->arrive[a] = 0;
        C->done = 0;
        C->iterations = 0;
        C->status = SUBSURF4D_OK;
        C->final_red = 0;
        C->bn = 0.0;
        C->rel_res = 0.0;
        C->tol = tol;
        C->max_iter = max_outer;
        C->outer = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *T.active = T.n_jobs;
        *T.pass = 0;
    }
}

// Colour-split copy of every padded cell of u^{resc;n-1} (its ghost layer is
// the Dirichlet data) into x, one thread per padded cell.
__global__ __launch_bounds__(kBlock) void kb_split_u(BTable T)
{
    for_runs(T.asm_start, nullptr, T.n_jobs, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        SS4_GLOBAL const double* u = gbl(static_cast<const double*>(J.u));
        SS4_GLOBAL double* xr = gbl(J.xr);
        SS4_GLOBAL double* xb = gbl(J.xb);
        const uint32_t npad = (uint32_t)J.npad;
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t p = item * kItem + threadIdx.x;
            if (p >= npad) continue;
            const uint32_t prow = fdiv(p, J.mg_p1);
            const int i = (int)(p - prow * (uint32_t)J.p1);
            const uint32_t t2 = fdiv(prow, J.mg_p2);
            const int j = (int)(prow - t2 * (uint32_t)J.p2);
            const uint32_t t3 = fdiv(t2, J.mg_p3);
            const int k = (int)(t2 - t3 * (uint32_t)J.p3);
            const int l = (int)t3;
            const uint32_t us = prow * (uint32_t)J.rsu + 1 + ((i - 1) >> 1);
            if (((i + j + k + l) & 1) == 0) xr[us] = u[p];
            else xb[us] = u[p];
        }
    });
}

// Store of a batched assembly output, non-temporal when NT.
template <bool NT, typename P, typename V>
__device__ __forceinline__ void kput(P* p, V v)
{
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Assembly of every job, frame-marching: a work item is 256 consecutive
// (i,j,k) positions of one frame, and each thread walks the frames l = 1..N4
// of its position.  The values of u at the position and its six x/y/z
// neighbours are kept for frames l-1, l and l+1 in registers (they are the
// cell's t-neighbours and t-diagonals), so per frame a thread loads the seven
// of frame l+1 and the twelve in-frame diagonals of frame l; the t-face G of
// the frame below is kept as well.  Writes the colour-split tiles, the BF16
// records, r/D of the initial iterate, and one partial of ||b||^2 and of the
// initial residual per wave and item (a job's partials do not depend on the
// rest of the batch).
// FAST: the -t face's q and 1/sqrt(eps^2 + q) are carried from the frame
// below, where the same thread formed them, from the same values in the same
// order, as its +t face (same bits), and the outputs are written with
// non-temporal stores, so they do not push the u rows that the neighbouring
// items are about to read out of L2.  MIXED: also the BF16 records and r/D
// of the initial iterate, which only the mixed-precision form reads.
template <bool FAST, bool MIXED>
__global__ __launch_bounds__(kBlock) void kb_assemble(BTable T)
{
    for_runs(T.int_start, nullptr, T.n_jobs, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        SS4_GLOBAL const double* u = gbl(static_cast<const double*>(J.u));
        SS4_GLOBAL const double* G = gbl(J.G);
        SS4_GLOBAL double* coef = gbl(J.coef);
        SS4_GLOBAL u32x4* c16 = gbl(reinterpret_cast<u32x4*>(J.c16));
        SS4_GLOBAL float* rf = gbl(J.rf);
        SS4_GLOBAL double* pa = gbl(J.part_a);
        SS4_GLOBAL double* pb = gbl(J.part_b);
        const uint32_t npad = (uint32_t)J.npad;
        const uint32_t nfr = (uint32_t)J.n1 * (uint32_t)J.n2 * (uint32_t)J.n3;
        const uint32_t sd[4] = {1u, (uint32_t)J.p1, (uint32_t)J.p1 * J.p2, (uint32_t)J.p1 * J.p2 * J.p3};
        const int nn[4] = {J.n1, J.n2, J.n3, J.n4};
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t qi = item * kItem + threadIdx.x;
            double acc_b = 0.0, acc_r = 0.0;
            if (qi < nfr) {
                const uint32_t r1 = fdiv(qi, J.mg_n1);
                const int i = (int)(qi - r1 * (uint32_t)J.n1) + 1;
                const uint32_t r2 = fdiv(r1, J.mg_n2);
                const int j = (int)(r1 - r2 * (uint32_t)J.n2) + 1;
                const int k = (int)r2 + 1;
                const uint32_t p0 = ((uint32_t)k * J.p2 + (uint32_t)j) * J.p1 + (uint32_t)i;   // frame 0
                // u at the position and its x/y/z neighbours: 0 itself, 1/2 -x/+x, 3/4 -y/+y, 5/6 -z/+z
                auto axis = [&](uint32_t q, double (&A)[7]) {
                    A[0] = u[q];
                    A[1] = u[q - sd[0]];
                    A[2] = u[q + sd[0]];
                    A[3] = u[q - sd[1]];
                    A[4] = u[q + sd[1]];
                    A[5] = u[q - sd[2]];
                    A[6] = u[q + sd[2]];
                };
                double Am[7], Ac[7], Ap[7];
                axis(p0, Am);
                axis(p0 + sd[3], Ac);
                double gt_below = G[3u * npad + p0];
                double tq = 0.0, trs = 0.0;            // the +t face of the frame below (FAST)
                for (int l = 1; l <= J.n4; ++l) {
                    const bool carried = FAST && l > 1;
                    const uint32_t p = p0 + (uint32_t)l * sd[3];
                    axis(p + sd[3], Ap);
                    double dxy[2][2], dxz[2][2], dyz[2][2];   // in-frame diagonals [-/+][-/+]
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const int sa = 2 * a - 1, sc = 2 * c - 1;
                            dxy[a][c] = u[p + sa * (int)sd[0] + sc * (int)sd[1]];
                            dxz[a][c] = u[p + sa * (int)sd[0] + sc * (int)sd[2]];
                            dyz[a][c] = u[p + sa * (int)sd[1] + sc * (int)sd[2]];
                        }
                    // u at p + (dx, dy, dz, dt), at most two offsets non-zero
                    auto wat = [&](int dx, int dy, int dz, int dt) -> double {
                        const int ax = dx ? (dx < 0 ? 1 : 2) : dy ? (dy < 0 ? 3 : 4) : dz ? (dz < 0 ? 5 : 6) : 0;
                        if (dt != 0) return dt < 0 ? Am[ax] : Ap[ax];
                        if ((dx != 0) + (dy != 0) + (dz != 0) <= 1) return Ac[ax];
                        if (dz == 0) return dxy[(dx + 1) / 2][(dy + 1) / 2];
                        if (dy == 0) return dxz[(dx + 1) / 2][(dz + 1) / 2];
                        return dyz[(dy + 1) / 2][(dz + 1) / 2];
                    };
                    auto w1 = [&](int d, int sg) {
                        return wat(d == 0 ? sg : 0, d == 1 ? sg : 0, d == 2 ? sg : 0, d == 3 ? sg : 0);
                    };
                    auto w2 = [&](int d, int sgd, int t, int sgt) {
                        return wat((d == 0 ? sgd : 0) + (t == 0 ? sgt : 0), (d == 1 ? sgd : 0) + (t == 1 ? sgt : 0),
                                   (d == 2 ? sgd : 0) + (t == 2 ? sgt : 0), (d == 3 ? sgd : 0) + (t == 3 ? sgt : 0));
                    };
                    const int colour = (i + j + k + l) & 1;
                    const int m = (i - 1) >> 1;
                    const double w0 = Ac[0];
                    const int idx[4] = {i, j, k, l};
                    double wm[4], wp[4], q[8];
#pragma unroll
                    for (int d = 0; d < 4; ++d) { wm[d] = w1(d, -1); wp[d] = w1(d, 1); }
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        const bool skip_m = d == 3 && carried;
                        const double gnm = (w0 - wm[d]) * J.inv_h;
                        const double gnp = (wp[d] - w0) * J.inv_h;
                        double qm = gnm * gnm, qp = gnp * gnp;
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            if (t == d) continue;
                            const double wpt = wp[t], wmt = wm[t];
                            const double dp_pt = w2(d, 1, t, 1), dp_mt = w2(d, 1, t, -1);
                            const double tp = ((wpt + dp_pt) - (wmt + dp_mt)) * (0.25 * J.inv_h);
                            qp += tp * tp;
                            if (!skip_m) {
                                const double dm_pt = w2(d, -1, t, 1), dm_mt = w2(d, -1, t, -1);
                                const double tm = ((dm_pt + wpt) - (dm_mt + wmt)) * (0.25 * J.inv_h);
                                qm += tm * tm;
                            }
                        }
                        q[2 * d] = skip_m ? tq : qm;
                        q[2 * d + 1] = qp;
                    }
                    double qs = 0.0;
#pragma unroll
                    for (int f = 0; f < 8; ++f) qs += q[f];
                    const double scale = J.th2 * sqrt(J.eps2 + qs / 8.0);
                    const double gt_here = G[3u * npad + p];
                    double c[8];
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        const double gm = d == 3 ? gt_below : G[(uint32_t)d * npad + p - sd[d]];
                        const double gp = d == 3 ? gt_here : G[(uint32_t)d * npad + p];
                        const double rm = (d == 3 && carried) ? trs : rsqrt(J.eps2 + q[2 * d]);
                        const double rp = rsqrt(J.eps2 + q[2 * d + 1]);
                        c[2 * d] = scale * gm * rm;
                        c[2 * d + 1] = scale * gp * rp;
                        if (d == 3) { tq = q[7]; trs = rp; }
                    }
                    gt_below = gt_here;
                    double D = 1.0, bfull = w0, off = 0.0;
#pragma unroll
                    for (int f = 0; f < 8; ++f) D += c[f];
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        off += c[2 * d] * wm[d] + c[2 * d + 1] * wp[d];
                        if (idx[d] == 1) bfull += c[2 * d] * wm[d];
                        if (idx[d] == nn[d]) bfull += c[2 * d + 1] * wp[d];
                    }
                    const double r0 = (w0 + off) - D * w0;
                    acc_b += bfull * bfull;
                    acc_r += r0 * r0;
                    const uint32_t irow = ((uint32_t)(l - 1) * J.n3 + (uint32_t)(k - 1)) * J.n2 + (uint32_t)(j - 1);
                    const uint32_t qf = irow * (uint32_t)J.half + m;
                    const uint32_t ci = bctile(J, colour, qf);
#pragma unroll
                    for (int f = 0; f < 8; ++f) kput<FAST>(&coef[ci + f * kTileSlots], c[f]);
                    kput<FAST>(&coef[ci + 8 * kTileSlots], w0);
                    if (MIXED) {
                        const double inv = 1.0 / D;
                        // scaled residual of the initial iterate: the first refinement pass starts from it
                        kput<FAST>(&rf[(uint32_t)colour * (uint32_t)J.ntq * kTileSlots + qf], (float)(r0 / D));
                        uint32_t hb[8];
#pragma unroll
                        for (int f = 0; f < 8; ++f) hb[f] = bf16_bits((float)(c[f] * inv));
                        const u32x4 rec = {hb[0] | (hb[1] << 16), hb[2] | (hb[3] << 16), hb[4] | (hb[5] << 16),
                                           hb[6] | (hb[7] << 16)};
                        kput<FAST>(&c16[(uint32_t)colour * (uint32_t)J.ntq * kTileSlots + qf], rec);
                    }
#pragma unroll
                    for (int e = 0; e < 7; ++e) { Am[e] = Ac[e]; Ac[e] = Ap[e]; }
                }
            }
            const double bb = wave_sum(acc_b);
            const double rr = wave_sum(acc_r);
            if ((threadIdx.x & 63) == 0) {
                pa[item * kWaves + (threadIdx.x >> 6)] = bb;
                pb[item * kWaves + (threadIdx.x >> 6)] = rr;
            }
        }
    });
}

// Per-job fixed-order reduction of the assembly partials (one block per job):
// ||b||_2 and the residual of iterate 0.
__global__ __launch_bounds__(kBlock) void kb_assemble_decide(BTable T)
{
    __shared__ double lds[4];
    for (int jb = blockIdx.x; jb < T.n_jobs; jb += gridDim.x) {
        const BJob& J = T.jobs[jb];
        const int64_t nfr = (int64_t)J.n1 * J.n2 * J.n3;
        const int np = (int)(kWaves * ((nfr + kItem - 1) / kItem));
        const double B2 = sum_partials(J.part_a, np, lds);
        const double R2 = sum_partials(J.part_b, np, lds);
        if (threadIdx.x == 0) {
            Ctrl* C = J.C;
            C->bn = sqrt(B2);
            const double R = sqrt(R2);
            C->rel_res = C->bn > 0.0 ? R / C->bn : R;
            if (!(R2 < INFINITY) || !(B2 < INFINITY)) { C->status = SUBSURF4D_ENONFINITE; C->done = 1; }
            else if (R <= C->tol * C->bn) C->done = 1;
            if (C->done) atomicSub(T.active, 1);
        }
        __syncthreads();
    }
}

// FP64 residual r = b - A x of the refinement, frame-marching: a work item is
// 256 consecutive slots qf of one frame's flat numbering, and each thread
// walks the frames l = 1..N4 of its slot for both colours, so the other
// colour's t-neighbours and one x-neighbour stay in registers.  Writes r/D
// (FP32, the rhs of the correction sweeps) and one partial sum of r^2 per
// wave and item; the partials of a job do not depend on the rest of the
// batch.  MIXED: r/D is written (the FP64 form only needs the sums).
template <bool MIXED>
__global__ __launch_bounds__(kBlock) void kb_residual(BTable T)
{
    for_runs(T.act_colf, T.act_jobs, *T.n_act, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const uint32_t sy = J.rsu, sz = (uint32_t)J.p2 * J.rsu, st = sz * (uint32_t)J.p3;
        const uint32_t nqf = (uint32_t)J.nqf;
        SS4_GLOBAL const double* coef = gbl(static_cast<const double*>(J.coef));
        SS4_GLOBAL float* rf = gbl(J.rf);
        SS4_GLOBAL double* pa = gbl(J.part_a);
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t qf = item * kItem + threadIdx.x;
            double acc = 0.0;
            if (qf < nqf) {
                const uint32_t r = fdiv(qf, J.mg_half);
                const int m = (int)(qf - r * (uint32_t)J.half);
                const uint32_t r2 = fdiv(r, J.mg_n2);
                const int j = (int)(r - r2 * (uint32_t)J.n2) + 1;
                const int k = (int)r2 + 1;
                const uint32_t u0 = ((uint32_t)k * J.p2 + (uint32_t)j) * J.rsu + 1 + m;   // row (j,k,l=0)
#pragma unroll
                for (int colour = 0; colour < 2; ++colour) {
                    SS4_GLOBAL const double* own = gbl(static_cast<const double*>(colour ? J.xb : J.xr));
                    SS4_GLOBAL const double* oth = gbl(static_cast<const double*>(colour ? J.xr : J.xb));
                    const uint32_t cb = (uint32_t)colour * (uint32_t)J.ntq * kTileSlots;
                    double Bm = oth[u0];
                    double Bc = oth[u0 + st];
                    for (int l = 1; l <= J.n4; ++l) {
                        const uint32_t ui = u0 + (uint32_t)l * st;
                        const double Bp = oth[ui + st];
                        const int par = (colour + j + k + l) & 1;
                        const int cnt = par ? (J.n1 + 1) >> 1 : J.n1 >> 1;
                        if (m < cnt) {
                            const uint32_t q = (uint32_t)(l - 1) * nqf + qf;
                            SS4_GLOBAL const double* cf = coef + bctile(J, colour, q);
                            const double c0 = cf[0], c1 = cf[kTileSlots], c2 = cf[2 * kTileSlots];
                            const double c3 = cf[3 * kTileSlots], c4 = cf[4 * kTileSlots];
                            const double c5 = cf[5 * kTileSlots], c6 = cf[6 * kTileSlots];
                            const double c7 = cf[7 * kTileSlots];
                            const double xo = oth[par ? ui - 1 : ui + 1];
                            double s = cf[8 * kTileSlots];
                            s += c0 * (par ? xo : Bc) + c1 * (par ? Bc : xo);
                            s += c2 * oth[ui - sy] + c3 * oth[ui + sy];
                            s += c4 * oth[ui - sz] + c5 * oth[ui + sz];
                            s += c6 * Bm + c7 * Bp;
                            const double D = ((((((((1.0 + c0) + c1) + c2) + c3) + c4) + c5) + c6) + c7);
                            const double res = s - D * own[ui];
                            acc += res * res;
                            if (MIXED) rf[cb + q] = (float)(res / D);
                        }
                        Bm = Bc;
                        Bc = Bp;
                    }
                }
            }
            const double ws = wave_sum(acc);
            if ((threadIdx.x & 63) == 0) pa[item * kWaves + (threadIdx.x >> 6)] = ws;
        }
    });
}

// Per-job fixed-order reduction of the residual partials and the refinement
// stopping rule (one block per unfinished job).
__global__ __launch_bounds__(kBlock) void kb_residual_decide(BTable T)
{
    __shared__ double lds[4];
    const int pass = *T.pass;
    const int na = *T.n_act;
    for (int a = blockIdx.x; a < na; a += gridDim.x) {
        const BJob& J = T.jobs[T.act_jobs[a]];
        const double R2 = sum_partials(J.part_a, (int)(kWaves * J.nitf), lds);
        if (threadIdx.x == 0) {
            Ctrl* C = J.C;
            const double R = sqrt(R2);
            C->rel_res = C->bn > 0.0 ? R / C->bn : R;
            C->outer = pass;
            if (!(R2 < INFINITY)) { C->status = SUBSURF4D_ENONFINITE; C->done = 1; }
            else if (R <= C->tol * C->bn) { C->status = SUBSURF4D_OK; C->done = 1; }
            else if (pass >= T.max_outer) { C->status = SUBSURF4D_NOT_CONVERGED; C->done = 1; }
            if (C->done) atomicSub(T.active, 1);
        }
        __syncthreads();
    }
}

// FP32 half-sweep of colour COLOR on the scaled correction system.
// The relaxed update of one cell of the scaled correction system, shared by
// both work shapes so that they give the same bits.
__device__ __forceinline__ float sweep_cell(u32x4 cw, float s, float xl, float xr, float ym, float yp, float zm,
                                            float zp, float tm, float tp, float om, float om1, float old)
{
    s += bf16_lo(cw.x) * xl + bf16_hi(cw.x) * xr;
    s += bf16_lo(cw.y) * ym + bf16_hi(cw.y) * yp;
    s += bf16_lo(cw.z) * zm + bf16_hi(cw.z) * zp;
    s += bf16_lo(cw.w) * tm + bf16_hi(cw.w) * tp;
    return om * s + om1 * old;
}

// FIRST (both shapes): the first iteration of a refinement pass, which
// starts from d = 0.  Its red half-sweep is d = omega*r/D (no coefficient or
// neighbour reads) and its black half-sweep takes the old d as 0 without
// reading it; both give the bits of the general form on a zero d, so no pass
// needs d cleared beforehand.

// FP32 half-sweep of colour COLOR, flat shape: a work item is 256
// consecutive q of one colour.
template <int COLOR, bool FIRST>
__global__ __launch_bounds__(kBlock) void kb_sweep(BTable T)
{
    const float om = T.omega, om1 = 1.0f - T.omega;
    for_runs(T.act_col, T.act_jobs, *T.n_act, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const uint32_t sy = J.rsu, sz = (uint32_t)J.p2 * J.rsu, st = sz * (uint32_t)J.p3;
        SS4_GLOBAL float* own = gbl(COLOR ? J.db : J.dr);
        SS4_GLOBAL const float* oth = gbl(static_cast<const float*>(COLOR ? J.dr : J.db));
        const uint32_t cb = (uint32_t)COLOR * (uint32_t)J.ntq * kTileSlots;
        SS4_GLOBAL const u32x4* c16 = gbl(reinterpret_cast<const u32x4*>(J.c16));
        SS4_GLOBAL const float* rf = gbl(static_cast<const float*>(J.rf));
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t q = item * kItem + threadIdx.x;
            Cell c;
            if (!bdecode(J, COLOR, q, c)) continue;
            const uint32_t ui = c.prow * J.rsu + 1 + c.m;
            if constexpr (FIRST && COLOR == 0) {
                own[ui] = om * rf[cb + q];
                continue;
            }
            own[ui] = sweep_cell(c16[cb + q], rf[cb + q], oth[ui - c.par], oth[ui + 1 - c.par], oth[ui - sy],
                                 oth[ui + sy], oth[ui - sz], oth[ui + sz], oth[ui - st], oth[ui + st], om, om1,
                                 FIRST ? 0.0f : own[ui]);
        }
    });
}

// FP32 half-sweep of colour COLOR, frame-marching shape: a work item is 256
// consecutive slots qf = ((k-1)*N2 + (j-1))*half + m of one frame's flat
// numbering, and each thread walks the frames l = 1..N4 of its slot (a 4D
// tile of 256 slots x N4 frames).  The other colour's values of the slot at
// l-1, l, l+1 stay in registers: they are the cell's t-neighbours and one of
// its x-neighbours.  Cell (j,k,l) of slot m has q = (l-1)*nqf + qf.
template <int COLOR, bool FIRST>
__global__ __launch_bounds__(kBlock) void kb_sweep_tm(BTable T)
{
    const float om = T.omega, om1 = 1.0f - T.omega;
    for_runs(T.act_colf, T.act_jobs, *T.n_act, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const uint32_t sy = J.rsu, sz = (uint32_t)J.p2 * J.rsu, st = sz * (uint32_t)J.p3;
        SS4_GLOBAL float* own = gbl(COLOR ? J.db : J.dr);
        SS4_GLOBAL const float* oth = gbl(static_cast<const float*>(COLOR ? J.dr : J.db));
        const uint32_t cb = (uint32_t)COLOR * (uint32_t)J.ntq * kTileSlots;
        SS4_GLOBAL const u32x4* c16 = gbl(reinterpret_cast<const u32x4*>(J.c16));
        SS4_GLOBAL const float* rf = gbl(static_cast<const float*>(J.rf));
        const uint32_t nqf = (uint32_t)J.nqf;
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t qf = item * kItem + threadIdx.x;
            if (qf >= nqf) continue;
            const uint32_t r = fdiv(qf, J.mg_half);
            const int m = (int)(qf - r * (uint32_t)J.half);
            const uint32_t r2 = fdiv(r, J.mg_n2);
            const int j = (int)(r - r2 * (uint32_t)J.n2) + 1;
            const int k = (int)r2 + 1;
            const uint32_t u0 = ((uint32_t)k * J.p2 + (uint32_t)j) * J.rsu + 1 + m;   // row (j,k,l=0)
            if constexpr (FIRST && COLOR == 0) {
                for (int l = 1; l <= J.n4; ++l) {
                    const int par = (COLOR + j + k + l) & 1;
                    const int cnt = par ? (J.n1 + 1) >> 1 : J.n1 >> 1;
                    if (m < cnt) own[u0 + (uint32_t)l * st] = om * rf[cb + (uint32_t)(l - 1) * nqf + qf];
                }
                continue;
            }
            float Bm = oth[u0];
            float Bc = oth[u0 + st];
            for (int l = 1; l <= J.n4; ++l) {
                const uint32_t ui = u0 + (uint32_t)l * st;
                const float Bp = oth[ui + st];
                const int par = (COLOR + j + k + l) & 1;
                const int cnt = par ? (J.n1 + 1) >> 1 : J.n1 >> 1;
                if (m < cnt) {
                    const uint32_t q = (uint32_t)(l - 1) * nqf + qf;
                    const float xo = oth[par ? ui - 1 : ui + 1];
                    own[ui] = sweep_cell(c16[cb + q], rf[cb + q], par ? xo : Bc, par ? Bc : xo, oth[ui - sy],
                                         oth[ui + sy], oth[ui - sz], oth[ui + sz], Bm, Bp, om, om1,
                                         FIRST ? 0.0f : own[ui]);
                }
                Bm = Bc;
                Bc = Bp;
            }
        }
    });
}

// FP64 half-sweep of colour COLOR on the step's system itself (batched FP64
// form), frame-marching shape as kb_sweep_tm: x <- omega*(b + sum_f c_f x_f)/D
// + (1-omega)*x on the colour-split iterate, whose ghost slots hold the
// Dirichlet data.  Same arithmetic as the single-job FP64 sweep.
template <int COLOR>
__global__ __launch_bounds__(kBlock) void kb_sweep64_tm(BTable T)
{
    const double om = T.omega64, om1 = 1.0 - T.omega64;
    for_runs(T.act_colf, T.act_jobs, *T.n_act, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const uint32_t sy = J.rsu, sz = (uint32_t)J.p2 * J.rsu, st = sz * (uint32_t)J.p3;
        SS4_GLOBAL double* own = gbl(COLOR ? J.xb : J.xr);
        SS4_GLOBAL const double* oth = gbl(static_cast<const double*>(COLOR ? J.xr : J.xb));
        SS4_GLOBAL const double* coef = gbl(static_cast<const double*>(J.coef));
        const uint32_t nqf = (uint32_t)J.nqf;
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t qf = item * kItem + threadIdx.x;
            if (qf >= nqf) continue;
            const uint32_t r = fdiv(qf, J.mg_half);
            const int m = (int)(qf - r * (uint32_t)J.half);
            const uint32_t r2 = fdiv(r, J.mg_n2);
            const int j = (int)(r - r2 * (uint32_t)J.n2) + 1;
            const int k = (int)r2 + 1;
            const uint32_t u0 = ((uint32_t)k * J.p2 + (uint32_t)j) * J.rsu + 1 + m;   // row (j,k,l=0)
            double Bm = oth[u0];
            double Bc = oth[u0 + st];
            for (int l = 1; l <= J.n4; ++l) {
                const uint32_t ui = u0 + (uint32_t)l * st;
                const double Bp = oth[ui + st];
                const int par = (COLOR + j + k + l) & 1;
                const int cnt = par ? (J.n1 + 1) >> 1 : J.n1 >> 1;
                if (m < cnt) {
                    const uint32_t q = (uint32_t)(l - 1) * nqf + qf;
                    SS4_GLOBAL const double* cf = coef + bctile(J, COLOR, q);
                    const double c0 = cf[0], c1 = cf[kTileSlots], c2 = cf[2 * kTileSlots];
                    const double c3 = cf[3 * kTileSlots], c4 = cf[4 * kTileSlots];
                    const double c5 = cf[5 * kTileSlots], c6 = cf[6 * kTileSlots];
                    const double c7 = cf[7 * kTileSlots];
                    const double xo = oth[par ? ui - 1 : ui + 1];
                    double sum = cf[8 * kTileSlots];
                    sum += c0 * (par ? xo : Bc) + c1 * (par ? Bc : xo);
                    sum += c2 * oth[ui - sy] + c3 * oth[ui + sy];
                    sum += c4 * oth[ui - sz] + c5 * oth[ui + sz];
                    sum += c6 * Bm + c7 * Bp;
                    const double D = ((((((((1.0 + c0) + c1) + c2) + c3) + c4) + c5) + c6) + c7);
                    own[ui] = om * (sum / D) + om1 * own[ui];
                }
                Bm = Bc;
                Bc = Bp;
            }
        }
    });
}

// x += d for unfinished jobs (the next pass's first iteration does not read d).
__global__ __launch_bounds__(kBlock) void kb_update(BTable T)
{
    for_runs(T.act_both, T.act_jobs, *T.n_act, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const uint32_t nit = (uint32_t)J.nit;
        for (uint32_t item = i0; item < i1; item += step) {
            const int colour = item >= nit ? 1 : 0;
            const uint32_t q = (item - (colour ? nit : 0u)) * kItem + threadIdx.x;
            Cell c;
            if (!bdecode(J, colour, q, c)) continue;
            const uint32_t ui = c.prow * J.rsu + 1 + c.m;
            SS4_GLOBAL double* x = gbl(colour ? J.xb : J.xr);
            SS4_GLOBAL float* d = gbl(colour ? J.db : J.dr);
            x[ui] += (double)d[ui];
        }
    });
}

// Compacted list of unfinished jobs and its item prefixes (one block; a
// fixed-order scan, so the list is in job order).
constexpr int kScan = 1024;
__global__ __launch_bounds__(kScan) void kb_compact(BTable T)
{
    __shared__ int s_cnt[kScan];
    __shared__ int64_t s_sum[kScan];
    __shared__ int64_t s_sumf[kScan];
    const int per = (T.n_jobs + kScan - 1) / kScan;
    const int lo = threadIdx.x * per;
    const int hi = lo + per < T.n_jobs ? lo + per : T.n_jobs;
    int cnt = 0;
    int64_t sum = 0, sumf = 0;
    for (int jb = lo; jb < hi; ++jb)
        if (!T.jobs[jb].C->done) { ++cnt; sum += T.jobs[jb].nit; sumf += T.jobs[jb].nitf; }
    s_cnt[threadIdx.x] = cnt;
    s_sum[threadIdx.x] = sum;
    s_sumf[threadIdx.x] = sumf;
    __syncthreads();
    const int tid = (int)threadIdx.x;
    for (int d = 1; d < kScan; d <<= 1) {            // inclusive Hillis-Steele scan
        const int c = tid >= d ? s_cnt[tid - d] : 0;
        const int64_t v = tid >= d ? s_sum[tid - d] : 0;
        const int64_t vf = tid >= d ? s_sumf[tid - d] : 0;
        __syncthreads();
        s_cnt[threadIdx.x] += c;
        s_sum[threadIdx.x] += v;
        s_sumf[threadIdx.x] += vf;
        __syncthreads();
    }
    int pos = s_cnt[threadIdx.x] - cnt;
    int64_t base = s_sum[threadIdx.x] - sum, basef = s_sumf[threadIdx.x] - sumf;
    for (int jb = lo; jb < hi; ++jb) {
        if (T.jobs[jb].C->done) continue;
        T.act_jobs[pos] = jb;
        T.act_col[pos] = base;
        T.act_both[pos] = 2 * base;
        T.act_colf[pos] = basef;
        ++pos;
        base += T.jobs[jb].nit;
        basef += T.jobs[jb].nitf;
    }
    if (threadIdx.x == kScan - 1) {
        const int na = s_cnt[kScan - 1];
        T.act_col[na] = s_sum[kScan - 1];
        T.act_both[na] = 2 * s_sum[kScan - 1];
        T.act_colf[na] = s_sumf[kScan - 1];
        *T.n_act = na;
    }
}

__global__ void kb_gather(BTable T)
{
    for (int jb = blockIdx.x * blockDim.x + threadIdx.x; jb < T.n_jobs; jb += gridDim.x * blockDim.x)
        T.out[jb] = *T.jobs[jb].C;
}

__global__ void kb_next_pass(BTable T)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *T.pass += 1;
}

// zero both corrections of every job (ghost slots included)
__global__ void kb_zero_d(BTable T)
{
    for (int jb = blockIdx.y; jb < T.n_jobs; jb += gridDim.y) {
        const BJob& J = T.jobs[jb];
        const int64_t n = J.nrow_pad * J.rsu;
        for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
            J.dr[q] = 0.0f;
            J.db[q] = 0.0f;
        }
    }
}

// x -> interior of the padded u, every job
__global__ __launch_bounds__(kBlock) void kb_unsplit(BTable T)
{
    for_runs(T.both_start, nullptr, T.n_jobs, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const uint32_t nit = (uint32_t)J.nit;
        SS4_GLOBAL double* u = gbl(J.u);
        for (uint32_t item = i0; item < i1; item += step) {
            const int colour = item >= nit ? 1 : 0;
            const uint32_t q = (item - (colour ? nit : 0u)) * kItem + threadIdx.x;
            Cell c;
            if (!bdecode(J, colour, q, c)) continue;
            const int i = 2 * c.m + 2 - (c.par ? 1 : 0);
            SS4_GLOBAL const double* x = gbl(static_cast<const double*>(colour ? J.xb : J.xr));
            u[c.prow * (uint32_t)J.p1 + i] = x[c.prow * J.rsu + 1 + c.m];
        }
    });
}

}  // namespace

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace carving of one job in the batched layout.
bool plan_batch_job(const int32_t n[4], int32_t nc, BJob* J, size_t* bytes)
{
    for (int d = 0; d < 4; ++d)
        if (n[d] < 1 || n[d] > (1 << 16)) return false;
    // windows: every per-job array stays below 4 GiB (32-bit byte offsets)
    if ((int64_t)(n[0] + 2) * (n[1] + 2) * (n[2] + 2) * (n[3] + 2) > kBatchMaxPadded) return false;
    BJob b{};
    b.n1 = n[0]; b.n2 = n[1]; b.n3 = n[2]; b.n4 = n[3];
    b.p1 = n[0] + 2; b.p2 = n[1] + 2; b.p3 = n[2] + 2; b.p4 = n[3] + 2;
    b.half = (n[0] + 1) / 2;
    b.rsu = b.half + 2;
    b.nc = nc;
    b.nrow_int = (int64_t)n[1] * n[2] * n[3];
    b.nrow_pad = (int64_t)b.p2 * b.p3 * b.p4;
    b.npad = (int64_t)b.p1 * b.nrow_pad;
    b.nint = (int64_t)n[0] * b.nrow_int;
    b.ncq = b.nrow_int * b.half;
    b.ntq = (b.ncq + kTileSlots - 1) / kTileSlots;
    b.nip = (b.npad + kItem - 1) / kItem;
    b.mg_half = fdiv_magic((uint32_t)b.half);
    b.mg_n1 = fdiv_magic((uint32_t)n[0]);
    b.mg_n2 = fdiv_magic((uint32_t)n[1]);
    b.mg_n3 = fdiv_magic((uint32_t)n[2]);
    b.mg_p1 = fdiv_magic((uint32_t)b.p1);
    b.mg_p2 = fdiv_magic((uint32_t)b.p2);
    b.mg_p3 = fdiv_magic((uint32_t)b.p3);
    b.nit = (b.ncq + kItem - 1) / kItem;
    b.nqf = (int64_t)n[1] * n[2] * b.half;
    b.nitf = (b.nqf + kItem - 1) / kItem;
    const int64_t parts = kWaves * (b.nip > 2 * b.nit ? b.nip : 2 * b.nit);
    size_t off = 0;
    auto take = [&](size_t nbytes) { const size_t o = off; off += al256(nbytes); return o; };
    const size_t o_ctrl = take(sizeof(Ctrl));
    const size_t o_ctrl2 = take(sizeof(Ctrl));
    const size_t o_pa = take(sizeof(double) * parts);
    const size_t o_pb = take(sizeof(double) * parts);
    const size_t o_ball = take(sizeof(double) * 2 * (size_t)(nc > 0 ? nc : 1));
    const size_t o_xr = take(sizeof(double) * b.nrow_pad * b.rsu);
    const size_t o_xb = take(sizeof(double) * b.nrow_pad * b.rsu);
    const size_t o_coef = take(sizeof(double) * 2 * b.ntq * kTileVals);
    const size_t o_c16 = take(16 * 2 * b.ntq * kTileSlots);
    const size_t o_rf = take(sizeof(float) * 2 * b.ntq * kTileSlots);
    const size_t o_dr = take(sizeof(float) * b.nrow_pad * b.rsu);
    const size_t o_db = take(sizeof(float) * b.nrow_pad * b.rsu);
    // offsets are stored as pointers relative to a null base until bound
    b.C = reinterpret_cast<Ctrl*>(o_ctrl);
    b.C2 = reinterpret_cast<Ctrl*>(o_ctrl2);
    b.part_a = reinterpret_cast<double*>(o_pa);
    b.part_b = reinterpret_cast<double*>(o_pb);
    b.ball = reinterpret_cast<double*>(o_ball);
    b.xr = reinterpret_cast<double*>(o_xr);
    b.xb = reinterpret_cast<double*>(o_xb);
    b.coef = reinterpret_cast<double*>(o_coef);
    b.c16 = reinterpret_cast<uint4*>(o_c16);
    b.rf = reinterpret_cast<float*>(o_rf);
    b.dr = reinterpret_cast<float*>(o_dr);
    b.db = reinterpret_cast<float*>(o_db);
    *J = b;
    *bytes = off;
    return true;
}

size_t batch_job_bytes(const int32_t n[4], int32_t nc)
{
    BJob J;
    size_t b = 0;
    return plan_batch_job(n, nc, &J, &b) ? b : 0;
}

size_t batch_table_bytes(int32_t n_jobs)
{
    const size_t nj = (size_t)(n_jobs > 0 ? n_jobs : 1);
    return al256(sizeof(BJob) * nj) + al256(sizeof(Ctrl) * nj) + 8 * al256(sizeof(int64_t) * (nj + 1)) +
           al256(sizeof(int) * nj) + 256;
}

namespace {

template <typename T>
T* rebase(void* ws, T* off) { return reinterpret_cast<T*>(static_cast<char*>(ws) + reinterpret_cast<size_t>(off)); }

}  // namespace

int bind_batch_job(const int32_t n[4], int32_t nc, void* ws, size_t ws_bytes, BJob* out)
{
    BJob J;
    size_t need = 0;
    if (!plan_batch_job(n, nc, &J, &need)) {
        set_error("batched job: unsupported grid (at most 2^25 padded cells)");
        return SUBSURF4D_ESHAPE;
    }
    if (ws_bytes < need) {
        set_error("batched job: workspace too small (see subsurf4d_batch_workspace_bytes)");
        return SUBSURF4D_EWORKSPACE;
    }
    J.C = rebase(ws, J.C);
    J.C2 = rebase(ws, J.C2);
    J.part_a = rebase(ws, J.part_a);
    J.part_b = rebase(ws, J.part_b);
    J.ball = rebase(ws, J.ball);
    J.xr = rebase(ws, J.xr);
    J.xb = rebase(ws, J.xb);
    J.coef = rebase(ws, J.coef);
    J.c16 = rebase(ws, J.c16);
    J.rf = rebase(ws, J.rf);
    J.dr = rebase(ws, J.dr);
    J.db = rebase(ws, J.db);
    *out = J;
    return 0;
}

// Graph capture is not allowed on the legacy default stream: a batched step
// called on it runs on a library-owned non-blocking stream (default priority,
// one per device), ordered after the caller's earlier work by an event; the
// call synchronises before it returns.
// batches with fewer work items per colour than this skip the sweep-shape
// tuning run (about 26 windows of 40^3 x 5 cells)
constexpr int64_t kTuneMinItems = 1 << 14;

hipStream_t side_stream()
{
    static std::mutex mu;
    static std::map<int, hipStream_t> streams;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(mu);
    auto it = streams.find(dev);
    if (it != streams.end()) return it->second;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
    streams[dev] = st;
    return st;
}

// Executable graph of one refinement pass, kept per (device, stream): the
// pass is captured on every call (host-side work only) and the kept
// executable is updated in place with the new capture's kernel arguments and
// launch sizes; it is instantiated anew only when the update is refused (a
// different number of launches: other m or precision).
template <typename F>
int pass_graph(hipStream_t s, F&& enqueue, hipGraphExec_t* out)
{
    static std::mutex mu;
    static std::map<std::pair<int, hipStream_t>, hipGraphExec_t> kept;
    int dev = 0;
    SS4_HIP(hipGetDevice(&dev));
    hipGraph_t graph = nullptr;
    SS4_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    enqueue();
    SS4_HIP(hipStreamEndCapture(s, &graph));
    std::lock_guard<std::mutex> g(mu);
    const auto key = std::make_pair(dev, s);
    auto it = kept.find(key);
    hipError_t e = hipSuccess;
    if (it != kept.end()) {
        hipGraphExecUpdateResult how = hipGraphExecUpdateError;
        hipGraphNode_t bad = nullptr;
        e = hipGraphExecUpdate(it->second, graph, &bad, &how);
        if (e != hipSuccess || how != hipGraphExecUpdateSuccess) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(it->second);
            kept.erase(it);
            it = kept.end();
        }
    }
    if (it == kept.end()) {
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(e, "batched: graph instantiation");
        }
        it = kept.emplace(key, exec).first;
    }
    (void)hipGraphDestroy(graph);
    *out = it->second;
    return 0;
}

int run_batch_step_on(const subsurf4d_batch_job* jobs, int n_jobs, const subsurf4d_step_params& sp,
                      subsurf4d_result* results, void* table, size_t table_bytes, hipStream_t s);

int run_batch_step(const subsurf4d_batch_job* jobs, int n_jobs, const subsurf4d_step_params& sp,
                   subsurf4d_result* results, void* table, size_t table_bytes, hipStream_t s)
{
    if (s != nullptr) return run_batch_step_on(jobs, n_jobs, sp, results, table, table_bytes, s);
    hipStream_t w = side_stream();
    if (!w) {
        set_error("batched step: could not create a stream");
        return SUBSURF4D_EDEVICE;
    }
    hipEvent_t ev;
    SS4_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(w, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return hip_fail(e, "batched step: stream ordering");
    return run_batch_step_on(jobs, n_jobs, sp, results, table, table_bytes, w);
}

int run_batch_step_on(const subsurf4d_batch_job* jobs, int n_jobs, const subsurf4d_step_params& sp,
                      subsurf4d_result* results, void* table, size_t table_bytes, hipStream_t s)
{
    // host-side descriptors
    std::vector<BJob> hj(n_jobs);
    std::vector<int64_t> asm_start(n_jobs + 1), int_start(n_jobs + 1), col_start(n_jobs + 1), both_start(n_jobs + 1),
        ball_start(n_jobs + 1);
    asm_start[0] = int_start[0] = col_start[0] = both_start[0] = ball_start[0] = 0;
    for (int q = 0; q < n_jobs; ++q) {
        const subsurf4d_batch_job& bj = jobs[q];
        BJob J;
        const int nc = sp.rescale ? bj.n_centres : 0;
        if (int rc = bind_batch_job(bj.grid.n, nc, bj.workspace, bj.workspace_bytes, &J)) return rc;
        J.th2 = sp.tau / (bj.grid.h * bj.grid.h);
        J.eps2 = sp.eps * sp.eps;
        J.inv_h = 1.0 / bj.grid.h;
        J.G = bj.G;
        J.u = bj.u;
        J.owner = bj.owner;
        J.centres = bj.centres;
        hj[q] = J;
        asm_start[q + 1] = asm_start[q] + J.nip;
        int_start[q + 1] = int_start[q] + ((int64_t)J.n1 * J.n2 * J.n3 + kItem - 1) / kItem;   // frame items
        col_start[q + 1] = col_start[q] + J.nit;
        both_start[q + 1] = both_start[q] + 2 * J.nit;
        ball_start[q + 1] = ball_start[q] + J.nc;
    }
    if (table_bytes < batch_table_bytes(n_jobs)) {
        set_error("batched step: table workspace too small (see subsurf4d_batch_table_bytes)");
        return SUBSURF4D_EWORKSPACE;
    }
    char* tb = static_cast<char*>(table);
    size_t off = 0;
    BTable T{};
    T.jobs = reinterpret_cast<BJob*>(tb + off); off += al256(sizeof(BJob) * n_jobs);
    T.out = reinterpret_cast<Ctrl*>(tb + off); off += al256(sizeof(Ctrl) * n_jobs);
    T.asm_start = reinterpret_cast<int64_t*>(tb + off); off += al256(sizeof(int64_t) * (n_jobs + 1));
    T.int_start = reinterpret_cast<int64_t*>(tb + off); off += al256(sizeof(int64_t) * (n_jobs + 1));
    T.col_start = reinterpret_cast<int64_t*>(tb + off); off += al256(sizeof(int64_t) * (n_jobs + 1));
    T.both_start = reinterpret_cast<int64_t*>(tb + off); off += al256(sizeof(int64_t) * (n_jobs + 1));
    T.ball_start = reinterpret_cast<int64_t*>(tb + off); off += al256(sizeof(int64_t) * (n_jobs + 1));
    T.act_col = reinterpret_cast<int64_t*>(tb + off); off += al256(sizeof(int64_t) * (n_jobs + 1));
    T.act_both = reinterpret_cast<int64_t*>(tb + off); off += al256(sizeof(int64_t) * (n_jobs + 1));
    T.act_colf = reinterpret_cast<int64_t*>(tb + off); off += al256(sizeof(int64_t) * (n_jobs + 1));
    T.act_jobs = reinterpret_cast<int*>(tb + off); off += al256(sizeof(int) * n_jobs);
    T.active = reinterpret_cast<int*>(tb + off);
    T.pass = T.active + 1;
    T.n_act = T.active + 2;
    T.n_jobs = n_jobs;
    const int m = sp.inner_sweeps;
    const bool fp64 = sp.precision == SUBSURF4D_FP64;
    T.max_outer = sp.max_iter / m > 1 ? sp.max_iter / m : 1;
    T.omega = (float)sp.omega;
    T.omega64 = sp.omega;
    SS4_HIP(hipMemcpyAsync(T.jobs, hj.data(), sizeof(BJob) * n_jobs, hipMemcpyHostToDevice, s));
    SS4_HIP(hipMemcpyAsync(T.asm_start, asm_start.data(), sizeof(int64_t) * (n_jobs + 1), hipMemcpyHostToDevice, s));
    SS4_HIP(hipMemcpyAsync(T.int_start, int_start.data(), sizeof(int64_t) * (n_jobs + 1), hipMemcpyHostToDevice, s));
    SS4_HIP(hipMemcpyAsync(T.col_start, col_start.data(), sizeof(int64_t) * (n_jobs + 1), hipMemcpyHostToDevice, s));
    SS4_HIP(hipMemcpyAsync(T.both_start, both_start.data(), sizeof(int64_t) * (n_jobs + 1), hipMemcpyHostToDevice, s));
    SS4_HIP(hipMemcpyAsync(T.ball_start, ball_start.data(), sizeof(int64_t) * (n_jobs + 1), hipMemcpyHostToDevice, s));

    // SUBSURF4D_KB_ASM=0 selects the assembly without the carried -t face and
    // with plain stores (same bits)
    const char* env_asm = getenv("SUBSURF4D_KB_ASM");
    const bool asm_fast = !(env_asm && env_asm[0] == '0');
    const void* kasm = asm_fast ? (fp64 ? reinterpret_cast<const void*>(&kb_assemble<true, false>)
                                        : reinterpret_cast<const void*>(&kb_assemble<true, true>))
                                : (fp64 ? reinterpret_cast<const void*>(&kb_assemble<false, false>)
                                        : reinterpret_cast<const void*>(&kb_assemble<false, true>));
    const int g_asm = resident_grid(kasm);
    const int g_res = resident_grid(fp64 ? reinterpret_cast<const void*>(&kb_residual<false>)
                                         : reinterpret_cast<const void*>(&kb_residual<true>));
    const int g_up = resident_grid(reinterpret_cast<const void*>(&kb_update));
    const dim3 g_zero(64, n_jobs < 65535 ? n_jobs : 65535);

    kb_init<<<(n_jobs + 255) / 256, 256, 0, s>>>(T, fp64 ? sp.tol : sp.refine_tol, T.max_outer);
    const int g_dec = n_jobs < 4096 ? n_jobs : 4096;
    kb_split_u<<<g_up, kBlock, 0, s>>>(T);
    if (asm_fast && fp64) kb_assemble<true, false><<<g_asm, kBlock, 0, s>>>(T);
    else if (asm_fast) kb_assemble<true, true><<<g_asm, kBlock, 0, s>>>(T);
    else if (fp64) kb_assemble<false, false><<<g_asm, kBlock, 0, s>>>(T);
    else kb_assemble<false, true><<<g_asm, kBlock, 0, s>>>(T);
    kb_assemble_decide<<<g_dec, kBlock, 0, s>>>(T);
    kb_compact<<<1, kScan, 0, s>>>(T);
    if (!fp64) kb_zero_d<<<g_zero, 256, 0, s>>>(T);
    SS4_LAUNCHED("batched: assemble");

    // Autotuner of the inner sweep's 4D tile shape and launch shape: the first
    // batch with a given signature (device, job count, items) times both work shapes (flat 256-cell items,
    // or 256-slot x N4-frame marching columns) at grids of 1, 2 and 4 times
    // the resident size on its own data and keeps the fastest.  Shape and grid
    // change only which thread updates which cell, never a job's arithmetic
    // (the red-black iterate does not depend on the order within a colour);
    // the corrections are zeroed again afterwards.  Flags can force a shape.
    int g_sw = 0, shape = 0;
    const int forced = (sp.flags & SUBSURF4D_FLAG_SWEEP_FLAT) ? 1 : (sp.flags & SUBSURF4D_FLAG_SWEEP_MARCH) ? 2 : 0;
    auto sweep_pair = [&](int shp, int g, bool first) {
        if (shp == 0) {
            if (first) {
                kb_sweep<0, true><<<g, kBlock, 0, s>>>(T);
                kb_sweep<1, true><<<g, kBlock, 0, s>>>(T);
            } else {
                kb_sweep<0, false><<<g, kBlock, 0, s>>>(T);
                kb_sweep<1, false><<<g, kBlock, 0, s>>>(T);
            }
        } else {
            if (first) {
                kb_sweep_tm<0, true><<<g, kBlock, 0, s>>>(T);
                kb_sweep_tm<1, true><<<g, kBlock, 0, s>>>(T);
            } else {
                kb_sweep_tm<0, false><<<g, kBlock, 0, s>>>(T);
                kb_sweep_tm<1, false><<<g, kBlock, 0, s>>>(T);
            }
        }
    };
    const int g64 = fp64 ? resident_grid(reinterpret_cast<const void*>(&kb_sweep64_tm<0>)) : 0;
    if (fp64) {
        // the FP64 sweep has one shape (frame-marching) at the resident grid
    } else if (forced) {
        shape = forced - 1;
        g_sw = shape == 0 ? resident_grid(reinterpret_cast<const void*>(&kb_sweep<0, false>))
                          : resident_grid(reinterpret_cast<const void*>(&kb_sweep_tm<0, false>));
    } else {
        static std::mutex mu;
        // the signature is coarse on purpose: batches whose job sets differ but
        // whose total work (half-octave buckets of the item count) and
        // cell-weighted mean frame count agree share one decision, so a
        // serving loop whose batch changes every step does not re-tune it;
        // small batches (where a tuning run would cost more than it can save)
        // take the frame-marching shape at the resident grid untimed
        static std::map<std::tuple<int, int, int>, std::pair<int, int>> tuned;
        int dev = 0;
        (void)hipGetDevice(&dev);
        double cells = 0.0, frames = 0.0;
        for (int q = 0; q < n_jobs; ++q) {
            cells += (double)hj[q].nint;
            frames += (double)hj[q].nint * hj[q].n4;
        }
        const int work_bucket = (int)std::floor(2.0 * std::log2((double)col_start[n_jobs] + 1.0));
        const int mean_frames = (int)std::lround(cells > 0.0 ? frames / cells : 1.0);
        const auto key = std::make_tuple(dev, work_bucket, mean_frames);
        if (col_start[n_jobs] < kTuneMinItems) {
            shape = 1;
            g_sw = resident_grid(reinterpret_cast<const void*>(&kb_sweep_tm<0, false>));
        } else {
            std::lock_guard<std::mutex> g(mu);
            auto it = tuned.find(key);
            if (it != tuned.end()) { shape = it->second.first; g_sw = it->second.second; }
        }
        if (!g_sw) {
            hipEvent_t e0, e1;
            SS4_HIP(hipEventCreate(&e0));
            SS4_HIP(hipEventCreate(&e1));
            float best = 1e30f;
            for (int shp = 0; shp < 2; ++shp) {
                const int res = shp == 0 ? resident_grid(reinterpret_cast<const void*>(&kb_sweep<0, false>))
                                         : resident_grid(reinterpret_cast<const void*>(&kb_sweep_tm<0, false>));
                for (int mult = 1; mult <= 4; mult *= 2) {
                    const int g = res * mult;
                    sweep_pair(shp, g, false);
                    SS4_HIP(hipEventRecord(e0, s));
                    for (int rep = 0; rep < 2; ++rep) sweep_pair(shp, g, false);
                    SS4_HIP(hipEventRecord(e1, s));
                    SS4_HIP(hipEventSynchronize(e1));
                    float ms = 0.f;
                    SS4_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (ms < best) { best = ms; g_sw = g; shape = shp; }
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            kb_zero_d<<<g_zero, 256, 0, s>>>(T);
            SS4_LAUNCHED("batched: tuning");
            std::lock_guard<std::mutex> g(mu);
            tuned[key] = std::make_pair(shape, g_sw);
        }
    }

    // one refinement pass = m inner iterations, update, FP64 residual of the
    // new iterate, per-job decision, compaction (the assembly supplied the
    // residual and the decision of the initial iterate).  FP64 form: m FP64
    // red-black iterations of the system itself, then the same residual,
    // decision and compaction (the stopping rule is tested every m
    // iterations).  A pass after every job has finished does no work, so
    // passes are enqueued in chunks and the host reads the number of
    // unfinished jobs once per chunk.
    const bool eager = (sp.flags & SUBSURF4D_FLAG_NO_GRAPH) != 0;
    auto enqueue_pass = [&]() {
        if (fp64) {
            for (int it = 0; it < m; ++it) {
                kb_sweep64_tm<0><<<g64, kBlock, 0, s>>>(T);
                kb_sweep64_tm<1><<<g64, kBlock, 0, s>>>(T);
            }
        } else {
            for (int it = 0; it < m; ++it) sweep_pair(shape, g_sw, it == 0);
            kb_update<<<g_up, kBlock, 0, s>>>(T);
        }
        kb_next_pass<<<1, 64, 0, s>>>(T);
        if (fp64) kb_residual<false><<<g_res, kBlock, 0, s>>>(T);
        else kb_residual<true><<<g_res, kBlock, 0, s>>>(T);
        kb_residual_decide<<<g_dec, kBlock, 0, s>>>(T);
        kb_compact<<<1, kScan, 0, s>>>(T);
    };
    hipGraphExec_t exec = nullptr;
    if (!eager) {
        int rcg = pass_graph(s, enqueue_pass, &exec);
        if (rcg) return rcg;
    }

    int active = n_jobs;
    SS4_HIP(hipMemcpyAsync(&active, T.active, sizeof(int), hipMemcpyDeviceToHost, s));
    SS4_HIP(hipStreamSynchronize(s));
    int passes = 0;
    int chunk = 2;
    int rc = 0;
    while (active > 0) {
        if (passes > T.max_outer + 1) {
            set_error("internal: batched refinement ended without a decision");
            rc = SUBSURF4D_EDEVICE;
            break;
        }
        hipError_t e = hipSuccess;
        for (int c = 0; c < chunk && e == hipSuccess; ++c) {
            if (eager) {
                enqueue_pass();
                e = hipGetLastError();
            } else {
                e = hipGraphLaunch(exec, s);
            }
        }
        if (e == hipSuccess) e = hipMemcpyAsync(&active, T.active, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { rc = hip_fail(e, "batched: refinement pass"); break; }
        passes += chunk;
        chunk = chunk < 8 ? 2 * chunk : 8;
    }
    if (rc) return rc;

    kb_unsplit<<<g_up, kBlock, 0, s>>>(T);
    if (sp.rescale && ball_start[n_jobs] > 0) {
        const int gb = (int)(ball_start[n_jobs] < 65536 ? ball_start[n_jobs] : 65536);
        kb_rescale<0><<<gb, kBlock, 0, s>>>(T, sp.ball_r);
        kb_rescale<1><<<gb, kBlock, 0, s>>>(T, sp.ball_r);
    }
    SS4_LAUNCHED("batched: unsplit / rescale");
    // gather the outcomes
    std::vector<Ctrl> hc(n_jobs);
    kb_gather<<<(n_jobs + 255) / 256, 256, 0, s>>>(T);
    SS4_HIP(hipMemcpyAsync(hc.data(), T.out, sizeof(Ctrl) * n_jobs, hipMemcpyDeviceToHost, s));
    SS4_HIP(hipStreamSynchronize(s));
    int worst = 0;
    for (int q = 0; q < n_jobs; ++q) {
        if (results) {
            results[q].status = hc[q].status;
            results[q].iterations = hc[q].outer * m;
            results[q].outer_iterations = hc[q].outer;
            results[q].reserved = 0;
            results[q].rel_residual = hc[q].rel_res;
            results[q].bnorm = hc[q].bn;
        }
        if (hc[q].status == SUBSURF4D_ENONFINITE) worst = SUBSURF4D_ENONFINITE;
        else if (hc[q].status == SUBSURF4D_NOT_CONVERGED && worst == 0) worst = SUBSURF4D_NOT_CONVERGED;
    }
    if (worst == SUBSURF4D_ENONFINITE) {
        set_error("batched step: a job hit a non-finite residual (see its result)");
        return SUBSURF4D_ENONFINITE;
    }
    return worst;
}

}  // namespace ss4
