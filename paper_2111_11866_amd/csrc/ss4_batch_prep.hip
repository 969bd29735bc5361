// Batched preparation of many windows: ball ownership, local thresholding,
// implicit zero-Neumann presmoothing, face edge detector G, initial function
// and local rescaling (Sec. 3.1, the implementation overview of Sec. 3.5) for
// every job of a batch with one sequence of launches.  Each step takes the
// same arithmetic as the single-job kernels of ss4_prepare.hip; only the work
// distribution differs:
//
// * cell-wise steps walk a global list of 256-cell work items of all jobs;
// * ball-wise steps (ownership, ball min/max, seeds) run one block per ball
//   of a global ball list;
// * the two heat solves of every job (I0 and I^TH) are independent systems,
//   each with its own stopping rule, decided per job in a fixed order; one
//   heat-solve iteration (red, black, residual, decision) is captured as a
//   HIP graph and replayed until every system has stopped.
//
// Scratch (I0, I^TH and the two smoothed images) is carved from the job's
// batched-step workspace, whose coefficient region is not live until the
// job's first step.
#include <climits>
#include <cmath>
#include <vector>

#include "ss4_batch.hpp"

namespace ss4 {

struct PTable {
    BJob* jobs;
    int4* out;            // per job: status / iterations of the I0 and I^TH heat solves
    int64_t* int_start;   // prefix of interior work items
    int64_t* col_start;   // prefix of one colour's work items (flat per-colour numbering)
    int64_t* pad_start;   // prefix of padded work items
    int64_t* ball_start;  // prefix of centres
    int64_t* seed_start;  // prefix of seeds
    int* active;          // heat-solve systems not finished
    int* pass;            // heat-solve iteration k
    int n_jobs;
    int max_iter;
    double a, omega, tol;
};

namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// interior cell (1-based) of a flat interior index q (x fastest)
struct ICell {
    int i, j, k, l;
};

__device__ __forceinline__ ICell idecode(const BJob& J, uint32_t q)
{
    ICell c;
    const uint32_t row = fdiv(q, J.mg_n1);
    c.i = (int)(q - row * (uint32_t)J.n1) + 1;
    const uint32_t r2 = fdiv(row, J.mg_n2);
    c.j = (int)(row - r2 * (uint32_t)J.n2) + 1;
    const uint32_t r3 = fdiv(r2, J.mg_n3);
    c.k = (int)(r2 - r3 * (uint32_t)J.n3) + 1;
    c.l = (int)r3 + 1;
    return c;
}

__device__ __forceinline__ uint32_t biidx(const BJob& J, int i, int j, int k, int l)
{
    return (((uint32_t)(l - 1) * J.n3 + (uint32_t)(k - 1)) * J.n2 + (uint32_t)(j - 1)) * J.n1 + (uint32_t)(i - 1);
}

__device__ __forceinline__ uint32_t bpidx(const BJob& J, int i, int j, int k, int l)
{
    return (((uint32_t)l * J.p3 + (uint32_t)k) * J.p2 + (uint32_t)j) * J.p1 + (uint32_t)i;
}

__device__ __forceinline__ uint32_t int_items(const BJob& J) { return (uint32_t)((J.nint + kItem - 1) / kItem); }

__global__ void kp_init(PTable T)
{
    for (int jb = blockIdx.x * blockDim.x + threadIdx.x; jb < T.n_jobs; jb += gridDim.x * blockDim.x) {
        for (int f = 0; f < 2; ++f) {
            Ctrl* C = f ? T.jobs[jb].C2 : T.jobs[jb].C;
            for (int a = 0; a < 4; ++a) C->arrive[a] = 0;
            C->done = 0;
            C->iterations = 0;
            C->status = SUBSURF4D_OK;
            C->final_red = 0;
            C->bn = 0.0;
            C->rel_res = 0.0;
            C->tol = T.tol;
            C->max_iter = T.max_iter;
            C->outer = 0;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *T.active = 2 * T.n_jobs;
        *T.pass = 0;
    }
}

// I0 = scale * image; owner and nearest-distance key reset
__global__ __launch_bounds__(kBlock) void kp_cast(PTable T, double scale)
{
    for_runs(T.int_start, nullptr, T.n_jobs, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const uint32_t n = (uint32_t)J.nint;
        int32_t* owner = const_cast<int32_t*>(J.owner);
        uint64_t* key = reinterpret_cast<uint64_t*>(J.S0);
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t q = item * kItem + threadIdx.x;
            if (q >= n) continue;
            double v;
            if (J.dtype == SUBSURF4D_U8) v = (double)static_cast<const uint8_t*>(J.image)[q];
            else if (J.dtype == SUBSURF4D_F32) v = (double)static_cast<const float*>(J.image)[q];
            else v = static_cast<const double*>(J.image)[q];
            J.I0[q] = __dmul_rn(scale, v);
            owner[q] = INT_MAX;
            key[q] = ~0ull;
        }
    });
}

// Ownership: pass 1 keeps the smallest squared distance to a containing
// centre per cell, pass 2 gives the cell to the lowest centre index at that
// distance (one block per ball of the global ball list).
template <int PASS>
__global__ __launch_bounds__(kBlock) void kp_owner(PTable T, double r)
{
    const int64_t total = T.ball_start[T.n_jobs];
    const double r2 = __dmul_rn(r, r);
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int jb = find_job(T.ball_start, T.n_jobs, w);
        const BJob& J = T.jobs[jb];
        const int m = (int)(w - T.ball_start[jb]);
        const subsurf4d_centre c = J.centres[m];
        int lo0, lo1, lo2, w0, w1;
        int64_t count;
        if (!bball(J, c, r, lo0, lo1, lo2, w0, w1, count)) continue;
        uint64_t* key = reinterpret_cast<uint64_t*>(J.S0);
        int32_t* owner = const_cast<int32_t*>(J.owner);
        for (uint32_t qq = threadIdx.x; qq < (uint32_t)count; qq += blockDim.x) {
            const uint32_t a = qq / (uint32_t)w0, b = a / (uint32_t)w1;
            const int i = lo0 + (int)(qq - a * (uint32_t)w0);
            const int j = lo1 + (int)(a - b * (uint32_t)w1);
            const int k = lo2 + (int)b;
            const double d2 = dist2_exact((double)(i - 1) - (double)c.x, (double)(j - 1) - (double)c.y,
                                          (double)(k - 1) - (double)c.z);
            if (!(d2 <= r2)) continue;
            const uint32_t cell = biidx(J, i, j, k, c.frame + 1);
            if (PASS == 1) {
                atomicMin((unsigned long long*)&key[cell], (unsigned long long)__double_as_longlong(d2));
            } else {
                if (key[cell] == (uint64_t)__double_as_longlong(d2)) atomicMin(&owner[cell], m);
            }
        }
    }
}

// alpha = min, beta = max of I0 over each ball (one block per ball)
__global__ __launch_bounds__(kBlock) void kp_ball_minmax(PTable T, double r)
{
    __shared__ double s_lo[4], s_hi[4];
    const int64_t total = T.ball_start[T.n_jobs];
    const double r2 = __dmul_rn(r, r);
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int jb = find_job(T.ball_start, T.n_jobs, w);
        const BJob& J = T.jobs[jb];
        const int m = (int)(w - T.ball_start[jb]);
        const subsurf4d_centre c = J.centres[m];
        int lo0, lo1, lo2, w0, w1;
        int64_t count;
        double lo = INFINITY, hi = -INFINITY;
        if (bball(J, c, r, lo0, lo1, lo2, w0, w1, count)) {
            for (uint32_t qq = threadIdx.x; qq < (uint32_t)count; qq += blockDim.x) {
                const uint32_t a = qq / (uint32_t)w0, b = a / (uint32_t)w1;
                const int i = lo0 + (int)(qq - a * (uint32_t)w0);
                const int j = lo1 + (int)(a - b * (uint32_t)w1);
                const int k = lo2 + (int)b;
                const double d2 = dist2_exact((double)(i - 1) - (double)c.x, (double)(j - 1) - (double)c.y,
                                              (double)(k - 1) - (double)c.z);
                if (!(d2 <= r2)) continue;
                const double v = J.I0[biidx(J, i, j, k, c.frame + 1)];
                lo = fmin(lo, v);
                hi = fmax(hi, v);
            }
        }
        lo = wave_min(lo);
        hi = wave_max(hi);
        if ((threadIdx.x & 63) == 0) { s_lo[threadIdx.x >> 6] = lo; s_hi[threadIdx.x >> 6] = hi; }
        __syncthreads();
        if (threadIdx.x == 0) {
            J.ball[2 * m] = fmin(fmin(s_lo[0], s_lo[1]), fmin(s_lo[2], s_lo[3]));
            J.ball[2 * m + 1] = fmax(fmax(s_hi[0], s_hi[1]), fmax(s_hi[2], s_hi[3]));
        }
        __syncthreads();
    }
}

// Cells without an owner get -1; local thresholding on owned cells.
__global__ __launch_bounds__(kBlock) void kp_threshold(PTable T, double lam)
{
    for_runs(T.int_start, nullptr, T.n_jobs, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const uint32_t n = (uint32_t)J.nint;
        int32_t* owner = const_cast<int32_t*>(J.owner);
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t q = item * kItem + threadIdx.x;
            if (q >= n) continue;
            const int m = owner[q];
            if (m == INT_MAX) {
                owner[q] = -1;
                J.ITH[q] = J.I0[q];
                continue;
            }
            const double a = J.ball[2 * m], b = J.ball[2 * m + 1];
            const double th = threshold_exact(lam, a, b);
            J.ITH[q] = (J.I0[q] >= th) ? b : a;
        }
    });
}

// Heat solve start: J = rhs for both systems and ||rhs||^2 per-wave partials.
__global__ __launch_bounds__(kBlock) void kp_lhe_start(PTable T)
{
    for_runs(T.int_start, nullptr, T.n_jobs, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const uint32_t n = (uint32_t)J.nint;
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t q = item * kItem + threadIdx.x;
            double b0 = 0.0, b1 = 0.0;
            if (q < n) {
                b0 = J.I0[q];
                b1 = J.ITH[q];
                J.S0[q] = b0;
                J.S1[q] = b1;
            }
            const double s0 = wave_sum(b0 * b0), s1 = wave_sum(b1 * b1);
            if ((threadIdx.x & 63) == 0) {
                J.part_a[item * kWaves + (threadIdx.x >> 6)] = s0;
                J.part_b[item * kWaves + (threadIdx.x >> 6)] = s1;
            }
        }
    });
}

// ||rhs||_2 of both systems (one block per job, fixed order)
__global__ __launch_bounds__(kBlock) void kp_lhe_bnorm(PTable T)
{
    __shared__ double lds[4];
    for (int jb = blockIdx.x; jb < T.n_jobs; jb += gridDim.x) {
        const BJob& J = T.jobs[jb];
        const int np = (int)(kWaves * int_items(J));
        const double B0 = sum_partials(J.part_a, np, lds);
        const double B1 = sum_partials(J.part_b, np, lds);
        if (threadIdx.x == 0) {
            J.C->bn = sqrt(B0);
            J.C2->bn = sqrt(B1);
        }
        __syncthreads();
    }
}

// Row P of the heat system (1 + a n_P) J_P - a sum_{interior nbrs} J_nbr = rhs_P
// (zero Neumann boundary): returns rhs_P + a sum_nbrs v_nbr and sets *D = 1 + a n_P.
__device__ __forceinline__ double lhe_row(const BJob& J, double a, const double* rhs, const double* v, uint32_t q,
                                         const ICell& c, double* D)
{
    const uint32_t sy = J.n1, sz = (uint32_t)J.n1 * J.n2, st = sz * (uint32_t)J.n3;
    double s = rhs[q];
    int cnt = 0;
    if (c.i > 1) { s += a * v[q - 1]; ++cnt; }
    if (c.i < J.n1) { s += a * v[q + 1]; ++cnt; }
    if (c.j > 1) { s += a * v[q - sy]; ++cnt; }
    if (c.j < J.n2) { s += a * v[q + sy]; ++cnt; }
    if (c.k > 1) { s += a * v[q - sz]; ++cnt; }
    if (c.k < J.n3) { s += a * v[q + sz]; ++cnt; }
    if (c.l > 1) { s += a * v[q - st]; ++cnt; }
    if (c.l < J.n4) { s += a * v[q + st]; ++cnt; }
    *D = 1.0 + a * cnt;
    return s;
}

// Residual partials of the unfinished systems.
__global__ __launch_bounds__(kBlock) void kp_lhe_residual(PTable T)
{
    const double a = T.a;
    for_runs(T.int_start, nullptr, T.n_jobs, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const bool run0 = !J.C->done, run1 = !J.C2->done;
        if (!run0 && !run1) return;
        const uint32_t n = (uint32_t)J.nint;
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t q = item * kItem + threadIdx.x;
            double r0 = 0.0, r1 = 0.0;
            if (q < n) {
                const ICell c = idecode(J, q);
                double D;
                if (run0) {
                    const double s = lhe_row(J, a, J.I0, J.S0, q, c, &D);
                    const double r = s - D * J.S0[q];
                    r0 = r * r;
                }
                if (run1) {
                    const double s = lhe_row(J, a, J.ITH, J.S1, q, c, &D);
                    const double r = s - D * J.S1[q];
                    r1 = r * r;
                }
            }
            const double s0 = wave_sum(r0), s1 = wave_sum(r1);
            if ((threadIdx.x & 63) == 0) {
                if (run0) J.part_a[item * kWaves + (threadIdx.x >> 6)] = s0;
                if (run1) J.part_b[item * kWaves + (threadIdx.x >> 6)] = s1;
            }
        }
    });
}

// Stopping rule of iteration k for each unfinished system (one block per job).
__global__ __launch_bounds__(kBlock) void kp_lhe_decide(PTable T)
{
    __shared__ double lds[4];
    const int k = *T.pass;
    for (int jb = blockIdx.x; jb < T.n_jobs; jb += gridDim.x) {
        const BJob& J = T.jobs[jb];
        const int np = (int)(kWaves * int_items(J));
        for (int f = 0; f < 2; ++f) {
            Ctrl* C = f ? J.C2 : J.C;
            if (C->done) continue;                          // uniform: read by the whole block
            const double R2 = sum_partials(f ? J.part_b : J.part_a, np, lds);
            if (threadIdx.x == 0) {
                const double R = sqrt(R2);
                C->rel_res = C->bn > 0.0 ? R / C->bn : R;
                C->iterations = k;
                if (!(R2 < INFINITY)) { C->status = SUBSURF4D_ENONFINITE; C->done = 1; }
                else if (R <= C->tol * C->bn) C->done = 1;
                else if (k >= C->max_iter) { C->status = SUBSURF4D_NOT_CONVERGED; C->done = 1; }
                if (C->done) atomicSub(T.active, 1);
            }
            __syncthreads();
        }
    }
}

// The heat solves run on colour-split copies: colour c's cells at c*ncq + h,
// h = row*half + m the flat per-colour numbering (cell i = 2m + 2 - par of the
// interior row).  In the other colour's half, a cell's x-neighbours are
// h - par and h + 1 - par, and its y-, z- and t-neighbours keep m in the
// adjacent row, plane and frame, so every access of a sweep is a contiguous
// run.  Slots past a row's last cell of a colour hold 0 and are never read.
__device__ __forceinline__ uint32_t heat_q(const BJob& J, const Cell& cc)
{
    return ((((uint32_t)cc.l - 1) * (uint32_t)J.n3 + ((uint32_t)cc.k - 1)) * (uint32_t)J.n2 + ((uint32_t)cc.j - 1)) *
               (uint32_t)J.n1 + (uint32_t)(2 * cc.m + 1 - cc.par);
}

template <int COLOR>
__global__ __launch_bounds__(kBlock) void kp_heat_split(PTable T)
{
    for_runs(T.col_start, nullptr, T.n_jobs, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const uint32_t ncq = (uint32_t)J.ncq;
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t h = item * kItem + threadIdx.x;
            if (h >= ncq) continue;
            Cell cc;
            double v0 = 0.0, v1 = 0.0;
            if (bdecode(J, COLOR, h, cc)) {
                const uint32_t q = heat_q(J, cc);
                v0 = J.I0[q];
                v1 = J.ITH[q];
            }
            const uint32_t o = COLOR * ncq + h;
            J.HR0[o] = v0; J.HJ0[o] = v0;
            J.HR1[o] = v1; J.HJ1[o] = v1;
        }
    });
}

// the split iterates back into the natural S0 / S1
template <int COLOR>
__global__ __launch_bounds__(kBlock) void kp_heat_merge(PTable T)
{
    for_runs(T.col_start, nullptr, T.n_jobs, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const uint32_t ncq = (uint32_t)J.ncq;
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t h = item * kItem + threadIdx.x;
            Cell cc;
            if (!bdecode(J, COLOR, h, cc)) continue;
            const uint32_t q = heat_q(J, cc);
            J.S0[q] = J.HJ0[COLOR * ncq + h];
            J.S1[q] = J.HJ1[COLOR * ncq + h];
        }
    });
}

// Row of cell h of colour COLOR on the split copies: returns rhs + a sum_nbrs
// (other colour, interior neighbours only) and sets *D = 1 + a n_P; the
// neighbours are summed in the order -x, +x, -y, +y, -z, +z, -t, +t.
template <int COLOR>
__device__ __forceinline__ double lhe_row_split(const BJob& J, double a, const double* __restrict__ R,
                                                const double* __restrict__ O, uint32_t h, const Cell& cc, double* D)
{
    const uint32_t sy = (uint32_t)J.half, sz = sy * (uint32_t)J.n2, st = sz * (uint32_t)J.n3;
    const int i = 2 * cc.m + 2 - cc.par;
    double s = R[h];
    int cnt = 0;
    if (i > 1) { s += a * O[h - cc.par]; ++cnt; }
    if (i < J.n1) { s += a * O[h + 1 - cc.par]; ++cnt; }
    if (cc.j > 1) { s += a * O[h - sy]; ++cnt; }
    if (cc.j < J.n2) { s += a * O[h + sy]; ++cnt; }
    if (cc.k > 1) { s += a * O[h - sz]; ++cnt; }
    if (cc.k < J.n3) { s += a * O[h + sz]; ++cnt; }
    if (cc.l > 1) { s += a * O[h - st]; ++cnt; }
    if (cc.l < J.n4) { s += a * O[h + st]; ++cnt; }
    *D = 1.0 + a * cnt;
    return s;
}

// SOR half-sweep of colour COLOR on the split copies of the unfinished
// systems, with the stopping-rule residual of its rows fused in (the iterate is
// that of the red-black pass counter p = *T.pass).  The red sweep of pass p
// forms the red rows of iterate p-1, rhs - A J before their update, and keeps
// iterate p-1's red values in R0 / R1; the black sweep of pass p forms the
// black rows of iterate p right after their update.  One partial of r^2 per
// wave and item: red items first, then black items.
template <int COLOR>
__global__ __launch_bounds__(kBlock) void kp_lhe_sweep(PTable T)
{
    const double a = T.a, om = T.omega, om1 = 1.0 - T.omega;
    for_runs(T.col_start, nullptr, T.n_jobs, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const bool run0 = !J.C->done, run1 = !J.C2->done;
        if (!run0 && !run1) return;
        const uint32_t ncq = (uint32_t)J.ncq;
        const uint32_t own = COLOR * ncq, oth = (1 - COLOR) * ncq;
        const uint32_t pbase = COLOR ? (uint32_t)J.nit : 0u;
        for (uint32_t item = i0; item < i1; item += step) {
            double r0 = 0.0, r1 = 0.0;
            const uint32_t h = item * kItem + threadIdx.x;
            Cell cc;
            if (bdecode(J, COLOR, h, cc)) {
                double D;
                if (run0) {
                    const double s = lhe_row_split<COLOR>(J, a, J.HR0 + own, J.HJ0 + oth, h, cc, &D);
                    double* W = J.HJ0 + own;
                    const double uold = W[h], unew = om * (s / D) + om1 * uold;
                    W[h] = unew;
                    const double r = s - D * (COLOR == 0 ? uold : unew);
                    r0 = r * r;
                    if (COLOR == 0) J.R0[h] = uold;
                }
                if (run1) {
                    const double s = lhe_row_split<COLOR>(J, a, J.HR1 + own, J.HJ1 + oth, h, cc, &D);
                    double* W = J.HJ1 + own;
                    const double uold = W[h], unew = om * (s / D) + om1 * uold;
                    W[h] = unew;
                    const double r = s - D * (COLOR == 0 ? uold : unew);
                    r1 = r * r;
                    if (COLOR == 0) J.R1[h] = uold;
                }
            }
            const double s0 = wave_sum(r0), s1 = wave_sum(r1);
            if ((threadIdx.x & 63) == 0) {
                if (run0) J.part_a[(pbase + item) * kWaves + (threadIdx.x >> 6)] = s0;
                if (run1) J.part_b[(pbase + item) * kWaves + (threadIdx.x >> 6)] = s1;
            }
        }
    });
}

// Stopping rule of iterate k = pass - 1 >= 1 (between the red and the black
// sweep of pass k+1): its red rows' partials come from that red sweep, its
// black rows' from the black sweep of pass k.  One block per job, fixed order.
__global__ __launch_bounds__(kBlock) void kp_lhe_decide_lag(PTable T)
{
    __shared__ double lds[4];
    const int k = *T.pass - 1;
    if (k < 1) return;                                      // iterate 0: decided by the full residual
    for (int jb = blockIdx.x; jb < T.n_jobs; jb += gridDim.x) {
        const BJob& J = T.jobs[jb];
        const int np = (int)(kWaves * 2 * J.nit);
        for (int f = 0; f < 2; ++f) {
            Ctrl* C = f ? J.C2 : J.C;
            if (C->done) continue;                          // uniform: read by the whole block
            const double R2 = sum_partials(f ? J.part_b : J.part_a, np, lds);
            if (threadIdx.x == 0) {
                const double R = sqrt(R2);
                C->rel_res = C->bn > 0.0 ? R / C->bn : R;
                C->iterations = k;
                if (!(R2 < INFINITY)) { C->status = SUBSURF4D_ENONFINITE; C->done = 1; }
                else if (R <= C->tol * C->bn) C->done = 1;
                else if (k >= C->max_iter) { C->status = SUBSURF4D_NOT_CONVERGED; C->done = 1; }
                if (C->done) atomicSub(T.active, 1);
            }
            __syncthreads();
        }
    }
}

// A system decided on iterate k >= 1 at pass k+1, whose red sweep had already
// moved its red cells on: put iterate k's red values back (red half of the
// split copy; the other slots are never read).
__global__ __launch_bounds__(kBlock) void kp_lhe_restore(PTable T)
{
    for_runs(T.col_start, nullptr, T.n_jobs, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const bool b0 = J.C->iterations >= 1, b1 = J.C2->iterations >= 1;
        if (!b0 && !b1) return;
        const uint32_t ncq = (uint32_t)J.ncq;
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t h = item * kItem + threadIdx.x;
            if (h >= ncq) continue;
            if (b0) J.HJ0[h] = J.R0[h];
            if (b1) J.HJ1[h] = J.R1[h];
        }
    });
}

__global__ void kp_next_pass(PTable T)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *T.pass += 1;
}

// the smoothed images become the right-hand sides of the next heat step
__global__ __launch_bounds__(kBlock) void kp_lhe_rotate(PTable T)
{
    for_runs(T.int_start, nullptr, T.n_jobs, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const uint32_t n = (uint32_t)J.nint;
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t q = item * kItem + threadIdx.x;
            if (q >= n) continue;
            J.I0[q] = J.S0[q];
            J.ITH[q] = J.S1[q];
        }
    });
}

// G on the 4 "+" faces of every padded cell (both images through face_q4)
__global__ __launch_bounds__(kBlock) void kp_face_g(PTable T, double K, double delta, double vartheta)
{
    for_runs(T.pad_start, nullptr, T.n_jobs, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const uint32_t npad = (uint32_t)J.npad;
        double* G = const_cast<double*>(J.G);
        const int n[4] = {J.n1, J.n2, J.n3, J.n4};
        const uint32_t stride[4] = {1u, (uint32_t)J.n1, (uint32_t)J.n1 * (uint32_t)J.n2,
                                    (uint32_t)J.n1 * (uint32_t)J.n2 * (uint32_t)J.n3};
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t p = item * kItem + threadIdx.x;
            if (p >= npad) continue;
            int c[4];
            const uint32_t row = fdiv(p, J.mg_p1);
            c[0] = (int)(p - row * (uint32_t)J.p1);
            const uint32_t r2 = fdiv(row, J.mg_p2);
            c[1] = (int)(row - r2 * (uint32_t)J.p2);
            const uint32_t r3 = fdiv(r2, J.mg_p3);
            c[2] = (int)(r2 - r3 * (uint32_t)J.p3);
            c[3] = (int)r3;
            uint32_t off[4][3];
#pragma unroll
            for (int d = 0; d < 4; ++d)
#pragma unroll
                for (int sh = -1; sh <= 1; ++sh) off[d][sh + 1] = (uint32_t)(clampi(c[d] + sh, 1, n[d]) - 1) * stride[d];
            double q0[4], q1[4];
            face_q4(J.S0, off, J.inv_h, q0);
            face_q4(J.S1, off, J.inv_h, q1);
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const double s = delta * sqrt(q0[d]) + vartheta * sqrt(q1[d]);
                G[(uint32_t)d * npad + p] = 1.0 / (1.0 + K * (s * s));
            }
        }
    });
}

// Initial function.  R <= 0: max over the frame's seeds of 1/(|X-s|+v) on
// interior cells, 0 on ghosts; R > 0: zero fill, then kp_init_scatter.
template <int DENSE>
__global__ __launch_bounds__(kBlock) void kp_init_u(PTable T, double v)
{
    for_runs(T.pad_start, nullptr, T.n_jobs, [&](int jb, uint32_t i0, uint32_t i1, uint32_t step) {
        const BJob J = T.jobs[jb];
        const uint32_t npad = (uint32_t)J.npad;
        for (uint32_t item = i0; item < i1; item += step) {
            const uint32_t p = item * kItem + threadIdx.x;
            if (p >= npad) continue;
            double best = 0.0;
            if (DENSE) {
                const uint32_t row = fdiv(p, J.mg_p1);
                const int i = (int)(p - row * (uint32_t)J.p1);
                const uint32_t r2 = fdiv(row, J.mg_p2);
                const int j = (int)(row - r2 * (uint32_t)J.p2);
                const uint32_t r3 = fdiv(r2, J.mg_p3);
                const int k = (int)(r2 - r3 * (uint32_t)J.p3);
                const int l = (int)r3;
                if (i >= 1 && i <= J.n1 && j >= 1 && j <= J.n2 && k >= 1 && k <= J.n3 && l >= 1 && l <= J.n4) {
                    bool any = false;
                    for (int m = 0; m < J.ns; ++m) {
                        const subsurf4d_centre c = J.seeds[m];
                        if (c.frame != l - 1) continue;
                        const double d2 = dist2_exact((double)(i - 1) - (double)c.x, (double)(j - 1) - (double)c.y,
                                                      (double)(k - 1) - (double)c.z);
                        const double val = __ddiv_rn(1.0, __dadd_rn(__dsqrt_rn(d2), v));
                        if (!any || val > best) best = val;
                        any = true;
                    }
                }
            }
            J.u[p] = best;
        }
    });
}

// R > 0: max(0, 1/(|X-s|+v) - 1/(R+v)) scattered over each seed's R-box (one
// block per seed; non-negative doubles order like their bit patterns).
__global__ __launch_bounds__(kBlock) void kp_init_scatter(PTable T, double v, double R)
{
    const int64_t total = T.seed_start[T.n_jobs];
    const double shift = __ddiv_rn(1.0, __dadd_rn(R, v));
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int jb = find_job(T.seed_start, T.n_jobs, w);
        const BJob& J = T.jobs[jb];
        const subsurf4d_centre c = J.seeds[w - T.seed_start[jb]];
        int lo0, lo1, lo2, w0, w1;
        int64_t count;
        if (!bball(J, c, R, lo0, lo1, lo2, w0, w1, count)) continue;
        for (uint32_t qq = threadIdx.x; qq < (uint32_t)count; qq += blockDim.x) {
            const uint32_t a = qq / (uint32_t)w0, b = a / (uint32_t)w1;
            const int i = lo0 + (int)(qq - a * (uint32_t)w0);
            const int j = lo1 + (int)(a - b * (uint32_t)w1);
            const int k = lo2 + (int)b;
            const double d2 = dist2_exact((double)(i - 1) - (double)c.x, (double)(j - 1) - (double)c.y,
                                          (double)(k - 1) - (double)c.z);
            const double val = __dsub_rn(__ddiv_rn(1.0, __dadd_rn(__dsqrt_rn(d2), v)), shift);
            if (val > 0.0)
                atomicMax((unsigned long long*)&J.u[bpidx(J, i, j, k, c.frame + 1)],
                          (unsigned long long)__double_as_longlong(val));
        }
    }
}

__global__ void kp_gather(PTable T)
{
    for (int jb = blockIdx.x * blockDim.x + threadIdx.x; jb < T.n_jobs; jb += gridDim.x * blockDim.x) {
        const BJob& J = T.jobs[jb];
        T.out[jb] = make_int4(J.C->status, J.C->iterations, J.C2->status, J.C2->iterations);
    }
}

}  // namespace

int run_batch_prepare_on(const subsurf4d_batch_prepare_job* jobs, int n_jobs, const subsurf4d_prepare_params& pp,
                         double v, double R, double ball_r, int32_t* statuses, void* table, size_t table_bytes,
                         hipStream_t s)
{
    std::vector<BJob> hj(n_jobs);
    std::vector<int64_t> int_start(n_jobs + 1, 0), col_start(n_jobs + 1, 0), pad_start(n_jobs + 1, 0),
        ball_start(n_jobs + 1, 0),
        seed_start(n_jobs + 1, 0);
    for (int q = 0; q < n_jobs; ++q) {
        const subsurf4d_batch_prepare_job& pj = jobs[q];
        BJob J;
        if (int rc = bind_batch_job(pj.grid.n, pj.n_centres, pj.workspace, pj.workspace_bytes, &J)) return rc;
        // scratch in the coefficient region: four interior FP64 fields, the
        // split rhs and iterate of both heat solves and their kept red values
        const size_t coef_bytes = sizeof(double) * 2 * (size_t)J.ntq * kTileVals;
        if (coef_bytes < sizeof(double) * (4 * (size_t)J.nint + 10 * (size_t)J.ncq)) {
            set_error("internal: batched preparation scratch does not fit");
            return SUBSURF4D_EDEVICE;
        }
        J.I0 = J.coef;
        J.ITH = J.I0 + J.nint;
        J.S0 = J.ITH + J.nint;
        J.S1 = J.S0 + J.nint;
        J.HR0 = J.S1 + J.nint;
        J.HR1 = J.HR0 + 2 * J.ncq;
        J.HJ0 = J.HR1 + 2 * J.ncq;
        J.HJ1 = J.HJ0 + 2 * J.ncq;
        J.R0 = J.HJ1 + 2 * J.ncq;
        J.R1 = J.R0 + J.ncq;
        J.inv_h = 1.0 / pj.grid.h;
        J.G = pj.G;
        J.u = pj.u;
        J.owner = pj.owner;
        J.centres = pj.centres;
        J.image = pj.image;
        J.dtype = pj.image_dtype;
        J.seeds = pj.seeds;
        J.ns = pj.n_seeds;
        hj[q] = J;
        int_start[q + 1] = int_start[q] + (J.nint + kItem - 1) / kItem;
        col_start[q + 1] = col_start[q] + J.nit;
        pad_start[q + 1] = pad_start[q] + J.nip;
        ball_start[q + 1] = ball_start[q] + J.nc;
        seed_start[q + 1] = seed_start[q] + J.ns;
    }
    if (table_bytes < batch_table_bytes(n_jobs)) {
        set_error("batched preparation: table workspace too small (see subsurf4d_batch_table_bytes)");
        return SUBSURF4D_EWORKSPACE;
    }
    char* tb = static_cast<char*>(table);
    size_t off = 0;
    PTable T{};
    T.jobs = reinterpret_cast<BJob*>(tb + off); off += al256(sizeof(BJob) * n_jobs);
    T.out = reinterpret_cast<int4*>(tb + off); off += al256(sizeof(Ctrl) * n_jobs);
    T.int_start = reinterpret_cast<int64_t*>(tb + off); off += al256(sizeof(int64_t) * (n_jobs + 1));
    T.col_start = reinterpret_cast<int64_t*>(tb + off); off += al256(sizeof(int64_t) * (n_jobs + 1));
    T.pad_start = reinterpret_cast<int64_t*>(tb + off); off += al256(sizeof(int64_t) * (n_jobs + 1));
    T.ball_start = reinterpret_cast<int64_t*>(tb + off); off += al256(sizeof(int64_t) * (n_jobs + 1));
    T.seed_start = reinterpret_cast<int64_t*>(tb + off); off += al256(sizeof(int64_t) * (n_jobs + 1));
    T.active = reinterpret_cast<int*>(tb + off);
    T.pass = T.active + 1;
    T.n_jobs = n_jobs;
    T.max_iter = pp.smooth_max_iter;
    T.tol = pp.smooth_tol;
    T.a = 0.0;
    T.omega = 1.0;
    SS4_HIP(hipMemcpyAsync(T.jobs, hj.data(), sizeof(BJob) * n_jobs, hipMemcpyHostToDevice, s));
    SS4_HIP(hipMemcpyAsync(T.int_start, int_start.data(), sizeof(int64_t) * (n_jobs + 1), hipMemcpyHostToDevice, s));
    SS4_HIP(hipMemcpyAsync(T.col_start, col_start.data(), sizeof(int64_t) * (n_jobs + 1), hipMemcpyHostToDevice, s));
    SS4_HIP(hipMemcpyAsync(T.pad_start, pad_start.data(), sizeof(int64_t) * (n_jobs + 1), hipMemcpyHostToDevice, s));
    SS4_HIP(hipMemcpyAsync(T.ball_start, ball_start.data(), sizeof(int64_t) * (n_jobs + 1), hipMemcpyHostToDevice, s));
    SS4_HIP(hipMemcpyAsync(T.seed_start, seed_start.data(), sizeof(int64_t) * (n_jobs + 1), hipMemcpyHostToDevice, s));

    const int g_cell = resident_grid(reinterpret_cast<const void*>(&kp_lhe_sweep<0>));
    const int g_job = n_jobs < 4096 ? n_jobs : 4096;
    const int64_t nballs = ball_start[n_jobs], nseeds = seed_start[n_jobs];
    const int g_ball = (int)(nballs < 65536 ? (nballs > 0 ? nballs : 1) : 65536);

    // ownership and local thresholding (A1)
    kp_init<<<(n_jobs + 255) / 256, 256, 0, s>>>(T);
    kp_cast<<<g_cell, kBlock, 0, s>>>(T, pp.image_scale);
    if (nballs > 0) {
        kp_owner<1><<<g_ball, kBlock, 0, s>>>(T, pp.ball_r);
        kp_owner<2><<<g_ball, kBlock, 0, s>>>(T, pp.ball_r);
        kp_ball_minmax<<<g_ball, kBlock, 0, s>>>(T, pp.ball_r);
    }
    kp_threshold<<<g_cell, kBlock, 0, s>>>(T, pp.lambda);
    SS4_LAUNCHED("batched preparation: ownership / threshold");

    // presmoothing (A2): both heat solves of every job
    int worst = 0;
    std::vector<int4> hout(n_jobs);
    if (pp.smooth_steps > 0) {
        const double h = jobs[0].grid.h;
        for (int q = 1; q < n_jobs; ++q)
            if (jobs[q].grid.h != h) {
                set_error("batched preparation: every job of a batch must have the same h");
                return SUBSURF4D_EINVAL;
            }
        T.a = pp.smooth_tau / (h * h);
        T.omega = pp.smooth_omega;
        if (!(T.omega > 0.0)) {
            const double rho = 8.0 * T.a / (1.0 + 8.0 * T.a);
            T.omega = 2.0 / (1.0 + sqrt(1.0 - rho * rho));
        }
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        SS4_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        // one red-black pass p: red sweep (red rows of iterate p-1), decision
        // on iterate p-1, black sweep (black rows of iterate p)
        kp_next_pass<<<1, 64, 0, s>>>(T);
        kp_lhe_sweep<0><<<g_cell, kBlock, 0, s>>>(T);
        kp_lhe_decide_lag<<<g_job, kBlock, 0, s>>>(T);
        kp_lhe_sweep<1><<<g_cell, kBlock, 0, s>>>(T);
        SS4_HIP(hipStreamEndCapture(s, &graph));
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        int rc = 0;
        for (int step = 0; step < pp.smooth_steps && rc == 0 && e == hipSuccess; ++step) {
            if (step > 0) kp_lhe_rotate<<<g_cell, kBlock, 0, s>>>(T);
            kp_init<<<(n_jobs + 255) / 256, 256, 0, s>>>(T);
            kp_lhe_start<<<g_cell, kBlock, 0, s>>>(T);
            kp_lhe_bnorm<<<g_job, kBlock, 0, s>>>(T);
            kp_lhe_residual<<<g_cell, kBlock, 0, s>>>(T);
            kp_lhe_decide<<<g_job, kBlock, 0, s>>>(T);
            kp_heat_split<0><<<g_cell, kBlock, 0, s>>>(T);
            kp_heat_split<1><<<g_cell, kBlock, 0, s>>>(T);
            e = hipGetLastError();
            int active = 2 * n_jobs, k = 0, chunk = 4;
            while (e == hipSuccess) {
                e = hipMemcpyAsync(&active, T.active, sizeof(int), hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess || active <= 0) break;
                // iterate k is decided at pass k+1, so up to smooth_max_iter + 1 passes
                if (k > pp.smooth_max_iter + 1) {
                    set_error("internal: batched heat solve ended without a decision");
                    rc = SUBSURF4D_EDEVICE;
                    break;
                }
                // passes past a system's decision leave it untouched
                for (int c = 0; c < chunk && k <= pp.smooth_max_iter + 1 && e == hipSuccess; ++c, ++k)
                    e = hipGraphLaunch(exec, s);
                chunk = chunk < 16 ? chunk * 2 : 16;
            }
            if (e == hipSuccess && rc == 0) {
                kp_lhe_restore<<<g_cell, kBlock, 0, s>>>(T);
                kp_heat_merge<0><<<g_cell, kBlock, 0, s>>>(T);
                kp_heat_merge<1><<<g_cell, kBlock, 0, s>>>(T);
                kp_gather<<<(n_jobs + 255) / 256, 256, 0, s>>>(T);
                e = hipMemcpyAsync(hout.data(), T.out, sizeof(int4) * n_jobs, hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                for (int q = 0; q < n_jobs && e == hipSuccess; ++q) {
                    const int st[2] = {hout[q].x, hout[q].z};
                    for (int f = 0; f < 2; ++f) {
                        if (st[f] == SUBSURF4D_ENONFINITE) worst = SUBSURF4D_ENONFINITE;
                        else if (st[f] == SUBSURF4D_NOT_CONVERGED && worst == 0) worst = SUBSURF4D_NOT_CONVERGED;
                        if (statuses && st[f] != 0 && (statuses[q] == 0 || st[f] < 0)) statuses[q] = st[f];
                    }
                }
            }
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "batched preparation: heat solve");
        if (rc) return rc;
        if (worst == SUBSURF4D_ENONFINITE) {
            set_error("non-finite residual in a batched presmoothing solve (see the job statuses)");
            return SUBSURF4D_ENONFINITE;
        }
    } else {
        // no smoothing: the edge detector sees I0 and I^TH themselves
        kp_lhe_start<<<g_cell, kBlock, 0, s>>>(T);
    }

    // edge detector on faces (A3), initial function and its local rescale
    kp_face_g<<<g_cell, kBlock, 0, s>>>(T, pp.K, pp.delta, pp.vartheta);
    if (R > 0.0) {
        kp_init_u<0><<<g_cell, kBlock, 0, s>>>(T, v);
        if (nseeds > 0)
            kp_init_scatter<<<(int)(nseeds < 65536 ? nseeds : 65536), kBlock, 0, s>>>(T, v, R);
    } else {
        kp_init_u<1><<<g_cell, kBlock, 0, s>>>(T, v);
    }
    if (ball_r >= 0.0 && nballs > 0) {
        BTable B{};
        B.jobs = T.jobs;
        B.ball_start = T.ball_start;
        B.n_jobs = n_jobs;
        kb_rescale<0><<<g_ball, kBlock, 0, s>>>(B, ball_r);
        kb_rescale<1><<<g_ball, kBlock, 0, s>>>(B, ball_r);
    }
    SS4_LAUNCHED("batched preparation: G / initial function");
    SS4_HIP(hipStreamSynchronize(s));
    return worst;
}

int run_batch_prepare(const subsurf4d_batch_prepare_job* jobs, int n_jobs, const subsurf4d_prepare_params& pp,
                      double v, double R, double ball_r, int32_t* statuses, void* table, size_t table_bytes,
                      hipStream_t s)
{
    if (statuses)
        for (int q = 0; q < n_jobs; ++q) statuses[q] = 0;
    if (s != nullptr) return run_batch_prepare_on(jobs, n_jobs, pp, v, R, ball_r, statuses, table, table_bytes, s);
    hipStream_t w = side_stream();
    if (!w) {
        set_error("batched preparation: could not create a stream");
        return SUBSURF4D_EDEVICE;
    }
    hipEvent_t ev;
    SS4_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(w, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return hip_fail(e, "batched preparation: stream ordering");
    return run_batch_prepare_on(jobs, n_jobs, pp, v, R, ball_r, statuses, table, table_bytes, w);
}

}  // namespace ss4
