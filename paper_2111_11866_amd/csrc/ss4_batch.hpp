// Batched windows: per-job descriptors, the device table, and the device
// helpers shared by the batched step and the batched preparation.
#pragma once

#include <hip/hip_runtime.h>

#include "ss4_internal.hpp"

namespace ss4 {

struct BJob {
    int n1, n2, n3, n4, p1, p2, p3, p4;
    int half, rsu, nc, pad0;
    int64_t nrow_int, nrow_pad, npad, nint;
    int64_t ncq;          // flat cells of one colour (incl. inactive slots)
    int64_t ntq;          // 128-tiles of one colour
    int64_t nip, nit;     // items over padded cells / over one colour
    int64_t nqf, nitf;    // one frame's flat cells of one colour, and its items (marching shape)
    uint64_t mg_half, mg_n1, mg_n2, mg_n3, mg_p1, mg_p2, mg_p3;   // ceil(2^63 / d) for the index divisions
    double th2, eps2, inv_h;
    const double* G;
    double* u;
    const int32_t* owner;
    const subsurf4d_centre* centres;
    double* xr;
    double* xb;
    double* coef;
    uint4* c16;
    float* rf;
    float* dr;
    float* db;
    double* part_a;       // per-wave partials (>= kWaves * max(nip, 2*nit))
    double* part_b;
    double* ball;         // mu, xi per centre (alpha, beta during preparation)
    Ctrl* C;
    Ctrl* C2;             // second control block (preparation: the I^TH heat solve)
    // preparation only
    const void* image;
    int dtype, ns;
    const subsurf4d_centre* seeds;
    double *I0, *ITH, *S0, *S1;   // interior FP64 scratch carved from the coefficient region
    double *HR0, *HR1, *HJ0, *HJ1;  // colour-split rhs and iterate of the two heat solves (same region)
    double *R0, *R1;              // red values of the last iterate of each heat solve (same region)
};

struct BTable {
    BJob* jobs;
    Ctrl* out;            // gathered per-job control blocks (n_jobs)
    int64_t* asm_start;   // prefix of nip
    int64_t* int_start;   // prefix of frame items ceil(n1 n2 n3 / kItem) (the assembly marches the frames)
    int64_t* col_start;   // prefix of nit
    int64_t* both_start;  // prefix of 2*nit
    int64_t* ball_start;  // prefix of nc
    int* active;          // jobs not finished
    int* pass;            // refinement pass counter (device, for graph replay)
    int* n_act;           // length of the compacted list of unfinished jobs
    int* act_jobs;        // unfinished jobs, in job order
    int64_t* act_col;     // prefix of nit over act_jobs
    int64_t* act_both;    // prefix of 2*nit over act_jobs
    int64_t* act_colf;    // prefix of nitf over act_jobs
    int n_jobs;
    int max_outer;
    float omega;          // mixed: relaxation of the FP32 correction sweeps
    int pad;
    double omega64;       // FP64: relaxation of the FP64 sweeps
};

size_t al256(size_t x);

// Workspace carving of one job in the batched layout (offsets from a null
// base until bound to the job's workspace with bind_batch_job).
bool plan_batch_job(const int32_t n[4], int32_t nc, BJob* J, size_t* bytes);
// Plan and bind one job's workspace; returns 0 or a SUBSURF4D_E* code.
int bind_batch_job(const int32_t n[4], int32_t nc, void* ws, size_t ws_bytes, BJob* J);
// Library-owned non-blocking stream of the current device (graph capture is
// not allowed on the legacy default stream).
hipStream_t side_stream();

namespace {


constexpr int kItem = 256;
constexpr int64_t kBatchMaxPadded = (int64_t)1 << 25;   // padded cells of one batched job
constexpr int kWaves = kItem / 64;      // per-wave partial sums per work item

#define SS4_GLOBAL __attribute__((address_space(1)))

// Global-memory view of a pointer: with a wave-uniform base the loads and
// stores take a 32-bit per-lane offset (every per-job array of the batched
// layout stays below 4 GiB).
template <typename T>
__device__ __forceinline__ SS4_GLOBAL T* gbl(T* p) { return (SS4_GLOBAL T*)p; }

// 16-byte record of the BF16 coefficients as a plain vector (HIP's uint4 is
// a class that does not bind to global-address-space references)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));


__device__ __forceinline__ int find_job(const int64_t* start, int n, int64_t w)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Work items of a global list (prefix `st` over `n` entries; entry a is job
// map[a], or a without a map) dealt to the blocks per XCD: the list is cut
// into one contiguous chunk per XCD (blocks are placed on the XCDs round
// robin), and in each round the blocks of one XCD take consecutive items of
// its chunk.  Rows that an item reads as neighbours (the rows beside it and
// the planes and frames before and after it) belong to items that the same
// XCD processes in the same or an adjacent round, so they are still in that
// XCD's L2.  Calls body(job, first, last, step) for each job's run of this
// block's items first, first+step, ... < last.
template <typename Body>
__device__ __forceinline__ void for_runs(const int64_t* st, const int* map, int n, Body&& body)
{
    const int64_t total = st[n];
    const int nx = (int)gridDim.x < kXcd ? (int)gridDim.x : kXcd;
    const int slots = (int)gridDim.x / nx;
    if ((int)blockIdx.x >= nx * slots) return;
    const int64_t chunk = (total + nx - 1) / nx;
    const int64_t beg = (int64_t)(blockIdx.x % nx) * chunk;
    const int64_t end = beg + chunk < total ? beg + chunk : total;
    int64_t w = beg + blockIdx.x / nx;
    if (w >= end) return;
    int a = find_job(st, n, w);
    while (w < end) {
        while (st[a + 1] <= w) ++a;
        const int64_t base = st[a];
        const int64_t stop = st[a + 1] < end ? st[a + 1] : end;
        body(map ? map[a] : a, (uint32_t)(w - base), (uint32_t)(stop - base), (uint32_t)slots);
        w += (stop - w + slots - 1) / slots * slots;      // first item of this block at or after stop
    }
}

__device__ __forceinline__ uint32_t bctile(const BJob& J, int colour, uint32_t q)
{
    return (((uint32_t)colour * (uint32_t)J.ntq + (q >> kTileShift)) * kTileFields) * kTileSlots +
           (q & (kTileSlots - 1));
}

// One cell of colour `colour` in the flat numbering: q = r*half + m with r the
// interior row (j,k,l) and m the slot; prow is the padded row index.
struct Cell {
    uint32_t prow;
    int m, j, k, l, par;
};

// decode flat q of colour `colour`: returns false for an inactive slot
__device__ __forceinline__ bool bdecode(const BJob& J, int colour, uint32_t q, Cell& c)
{
    if (q >= (uint32_t)J.ncq) return false;
    const uint32_t r = fdiv(q, J.mg_half);
    c.m = (int)(q - r * (uint32_t)J.half);
    const uint32_t r2 = fdiv(r, J.mg_n2);
    c.j = (int)(r - r2 * (uint32_t)J.n2) + 1;
    const uint32_t r3 = fdiv(r2, J.mg_n3);
    c.k = (int)(r2 - r3 * (uint32_t)J.n3) + 1;
    c.l = (int)r3 + 1;
    c.par = (colour + c.j + c.k + c.l) & 1;
    c.prow = ((uint32_t)c.l * (uint32_t)J.p3 + (uint32_t)c.k) * (uint32_t)J.p2 + (uint32_t)c.j;
    const int cnt = c.par ? (J.n1 + 1) >> 1 : J.n1 >> 1;
    return c.m < cnt;
}

// local rescaling of every job: one block per ball (global ball list)
__device__ __forceinline__ bool bball(const BJob& J, const subsurf4d_centre& c, double r, int& lo0, int& lo1, int& lo2,
                                      int& w0, int& w1, int64_t& count)
{
    if (c.frame < 0 || c.frame >= J.n4) return false;
    const double cc[3] = {(double)c.x, (double)c.y, (double)c.z};
    const int n[3] = {J.n1, J.n2, J.n3};
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        int v = (int)floor(cc[a] - r);
        lo[a] = v < 1 ? 1 : (v > n[a] ? n[a] : v);
        v = (int)ceil(cc[a] + r) + 2;
        hi[a] = v < 1 ? 1 : (v > n[a] ? n[a] : v);
    }
    lo0 = lo[0]; lo1 = lo[1]; lo2 = lo[2];
    w0 = hi[0] - lo[0] + 1;
    w1 = hi[1] - lo[1] + 1;
    count = (int64_t)w0 * w1 * (hi[2] - lo[2] + 1);
    return true;
}

template <int PHASE>
__global__ __launch_bounds__(kBlock) void kb_rescale(BTable T, double r)
{
    __shared__ double s_lo[4], s_hi[4];
    const int64_t total = T.ball_start[T.n_jobs];
    const double r2 = [&] {
#pragma clang fp contract(off)
        return r * r;
    }();
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int jb = find_job(T.ball_start, T.n_jobs, w);
        const BJob& J = T.jobs[jb];
        const int mball = (int)(w - T.ball_start[jb]);
        const subsurf4d_centre c = J.centres[mball];
        int lo0, lo1, lo2, w0, w1;
        int64_t count;
        const bool ok = bball(J, c, r, lo0, lo1, lo2, w0, w1, count);
        double mn = INFINITY, mx = -INFINITY, span = 0.0, mu = 0.0;
        if (PHASE == 1 && ok) {
            mu = J.ball[2 * mball];
            span = J.ball[2 * mball + 1] - mu;
        }
        if (ok && !(PHASE == 1 && !(span >= 1e-12))) {
            for (int64_t qq = threadIdx.x; qq < count; qq += blockDim.x) {
                const int i = lo0 + (int)(qq % w0);
                const int64_t q2 = qq / w0;
                const int j = lo1 + (int)(q2 % w1);
                const int k = lo2 + (int)(q2 / w1);
                const double d2 = dist2_exact((double)(i - 1) - (double)c.x, (double)(j - 1) - (double)c.y,
                                              (double)(k - 1) - (double)c.z);
                if (!(d2 <= r2)) continue;
                const int l = c.frame + 1;
                const int64_t p = (((int64_t)l * J.p3 + k) * J.p2 + j) * J.p1 + i;
                if (PHASE == 0) {
                    const double v = J.u[p];
                    mn = fmin(mn, v);
                    mx = fmax(mx, v);
                } else {
                    const int64_t ii = (((int64_t)(l - 1) * J.n3 + (k - 1)) * J.n2 + (j - 1)) * J.n1 + (i - 1);
                    if (J.owner[ii] == mball) J.u[p] = (J.u[p] - mu) / span;
                }
            }
        }
        if (PHASE == 0) {
            mn = wave_min(mn);
            mx = wave_max(mx);
            if ((threadIdx.x & 63) == 0) { s_lo[threadIdx.x >> 6] = mn; s_hi[threadIdx.x >> 6] = mx; }
            __syncthreads();
            if (threadIdx.x == 0) {
                J.ball[2 * mball] = fmin(fmin(s_lo[0], s_lo[1]), fmin(s_lo[2], s_lo[3]));
                J.ball[2 * mball + 1] = fmax(fmax(s_hi[0], s_hi[1]), fmax(s_hi[2], s_hi[3]));
            }
            __syncthreads();
        }
    }
}

}  // namespace
}  // namespace ss4
