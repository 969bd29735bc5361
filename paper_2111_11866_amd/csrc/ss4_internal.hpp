// Internal host-side interface between the C ABI and the kernel launchers.
#pragma once

#include <string>

#include "ss4_common.hpp"

namespace ss4 {

// Carving of the caller's workspace.  A small region (control block, per-block
// partials, per-ball scalars) is followed by a large region that the
// preparation and the time step use at different times.
struct WsPlan {
    Layout L;
    int32_t n_centres = 0;
    int32_t precision = 0;
    int64_t max_grid = 0;    // entries of each per-block partial array
    size_t ctrl = 0, part_a = 0, part_b = 0, balls = 0, big = 0;
    // time step
    size_t ured0 = 0, ured1 = 0, ublack = 0, coef = 0, rhs = 0;
    // mixed precision (inside the step region)
    size_t coef16 = 0, rf32 = 0, dred = 0, dblack = 0;
    // preparation
    size_t I0 = 0, ITH = 0, S0 = 0, S1 = 0;
    size_t HR = 0, HJ = 0, R = 0;   // heat solve: colour-split rhs and iterate, red values kept by the sweeps
    size_t step_bytes = 0, prep_bytes = 0, total = 0;
};

bool plan_workspace(const int32_t n[4], int32_t n_centres, int32_t precision, WsPlan* P);

template <typename T>
inline T* ws_ptr(void* ws, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(ws) + off); }

// Every launcher returns 0 or a negative SUBSURF4D_* status and sets the
// thread-local error text on failure.
void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define SS4_HIP(call)                                       \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return ss4::hip_fail(e_, #call); \
    } while (0)

#define SS4_LAUNCHED(what)                                  \
    do {                                                    \
        hipError_t e_ = hipGetLastError();                  \
        if (e_ != hipSuccess) return ss4::hip_fail(e_, what); \
    } while (0)

// Largest grid whose blocks are all resident at once on the current device
// (occupancy x compute units, a multiple of kXcd, at most kGridCap), so a
// grid-stride kernel never runs a partial second round of blocks.
int resident_grid(const void* kernel);
int resident_grid_bs(const void* kernel, int block);   // the same for blocks of `block` threads
// SUBSURF4D_SWEEP_GRID (percent of the resident grid, else dflt), read per solve
int sweep_grid_percent(int dflt);

// preparation (prepare.hip)
int run_prepare(const WsPlan& P, double h, const void* image, int dtype,
                const subsurf4d_centre* centres, int nc, const subsurf4d_prepare_params& pp,
                double* G, int32_t* owner, void* ws, hipStream_t s);
int run_init_u(const Layout& L, const subsurf4d_centre* seeds, int ns, double v, double R,
               double* u, hipStream_t s);
int run_rescale(const WsPlan& P, const subsurf4d_centre* centres, int nc, double r,
                const int32_t* owner, double* u, void* ws, hipStream_t s);

// time step and solve (solve.hip)
int run_assemble_export(const Layout& L, double h, const double* G, const double* u,
                        const subsurf4d_step_params& sp, double* coef, double* b, hipStream_t s);
// ub: padded array whose ghost layer holds the new level's Dirichlet data
// (NULL: u's own ghost layer serves both as gradient data and Dirichlet data)
int run_step(const WsPlan& P, double h, const double* G, const double* ub, const subsurf4d_centre* centres,
             int nc, const int32_t* owner, double* u, const subsurf4d_step_params& sp,
             subsurf4d_result* res, void* ws, hipStream_t s);
int run_solve(const WsPlan& P, const double* coef, const double* b, double* u,
              const subsurf4d_step_params& sp, subsurf4d_result* res, void* ws, hipStream_t s);

// the red-black iteration on a loaded system (solve.hip); used by step/solve
int run_sor_loop(const WsPlan& P, const subsurf4d_step_params& sp, void* ws, hipStream_t s,
                 subsurf4d_result* res);
int run_unsplit(const WsPlan& P, double* u, void* ws, hipStream_t s);
int launch_assembly(const WsPlan& P, double h, const double* G, const double* w, const double* ub,
                    const subsurf4d_step_params& sp, void* coef16, void* ws, hipStream_t s);
int run_copy_probe(const void* src, void* dst, size_t bytes, int reps, double* ms, hipStream_t s);
int stream_probe_grid(size_t bytes);
int run_stream_probe(const void* src, void* dst, size_t bytes, int reads, int writes, int reps, double* ms,
                     hipStream_t s);

// batched windows (batch.hip)
size_t batch_job_bytes(const int32_t n[4], int32_t nc);
size_t batch_table_bytes(int32_t n_jobs);
int run_batch_prepare(const subsurf4d_batch_prepare_job* jobs, int n_jobs, const subsurf4d_prepare_params& pp,
                      double v, double R, double ball_r, int32_t* statuses, void* table, size_t table_bytes,
                      hipStream_t s);
int run_batch_step(const subsurf4d_batch_job* jobs, int n_jobs, const subsurf4d_step_params& sp,
                   subsurf4d_result* results, void* table, size_t table_bytes, hipStream_t s);

// cell tracking (track.hip)
constexpr int64_t kTrackTableEntries = (int64_t)1 << 24;   // overlap table entries (at least)
size_t track_workspace_bytes(const int32_t n[4], int32_t capacity);
int run_track(const int32_t n[4], const double* u, double level, int32_t* lab, int32_t* d2, subsurf4d_cell* cells,
              int32_t capacity, int32_t* n_cells, void* ws, hipStream_t s);
int run_track_join(const int32_t n[4], subsurf4d_cell* cells, int32_t nc, double radius);

// mixed precision (mixed.hip)
int run_mixed_solve(const WsPlan& P, double h, const double* G, const double* w, const double* ub,
                    const subsurf4d_step_params& sp, subsurf4d_result* res, void* ws,
                    hipStream_t s);

}  // namespace ss4

namespace ss4 {

// Optional HIP-event timing of the red-black sweep chunks (enabled through
// subsurf4d_timing).  Events are recorded on the stream the sweeps run on.
struct TimingTotals {
    double sweep_ms = 0.0;        // summed duration of sweep chunks
    int64_t sweep_launches = 0;   // sweep launches that did work
    int64_t voxel_updates = 0;    // iterations x interior cells
    int64_t solves = 0;
};
bool timing_enabled();
void timing_add(double ms, int64_t launches, int64_t updates);

class SweepTimer {
public:
    explicit SweepTimer(hipStream_t s) : s_(s), on_(timing_enabled())
    {
        if (on_) {
            on_ = hipEventCreate(&a_) == hipSuccess && hipEventCreate(&b_) == hipSuccess;
        }
    }
    ~SweepTimer()
    {
        if (a_) (void)hipEventDestroy(a_);
        if (b_) (void)hipEventDestroy(b_);
    }
    hipEvent_t end_event() const { return on_ ? b_ : nullptr; }
    void begin() { if (on_) (void)hipEventRecord(a_, s_); }
    void end() { if (on_) (void)hipEventRecord(b_, s_); }
    void collect()
    {
        if (!on_) return;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, a_, b_) == hipSuccess) ms_ += ms;
    }
    void account(int64_t launches, int64_t updates)
    {
        if (on_) timing_add(ms_, launches, updates);
    }

private:
    hipStream_t s_;
    bool on_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
    double ms_ = 0.0;
};

// floor(n / d) for n < 2^31 with M = fdiv_magic(d) = ceil(2^63 / d): n*M/2^63
// exceeds n/d by less than 2^-32, and the fractional part of n/d is at most
// 1 - 1/d, so the floor is exact for every d < 2^32.
inline uint64_t fdiv_magic(uint32_t d) { return (((uint64_t)1 << 63) + d - 1) / d; }

__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint64_t M)
{
    const uint64_t lo = (uint64_t)n * (uint32_t)M;
    const uint64_t mid = (uint64_t)n * (uint32_t)(M >> 32) + (lo >> 32);
    return (uint32_t)(mid >> 31);
}

// Squared reduced-diamond-cell gradients of v on the four "+" faces of one cell
// (Sec. 3.2.2: normal difference over h, tangential ones as the mean of the
// two cells' central differences), with the image taken as its nearest
// interior value outside the box.  off[d][s + 1] is the offset along axis d of
// the clamped coordinate c_d + s, s in {-1, 0, 1}; the 27 values the four
// faces share are loaded once.
template <typename IDX>
__device__ __forceinline__ void face_q4(const double* __restrict__ v, const IDX (&off)[4][3], double inv_h,
                                        double (&q)[4])
{
    auto at = [&](int s0, int s1, int s2, int s3) {
        return v[off[0][s0 + 1] + off[1][s1 + 1] + off[2][s2 + 1] + off[3][s3 + 1]];
    };
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int e0 = d == 0, e1 = d == 1, e2 = d == 2, e3 = d == 3;
        const double g = (at(e0, e1, e2, e3) - at(0, 0, 0, 0)) * inv_h;
        double acc = g * g;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t == d) continue;
            const int f0 = t == 0, f1 = t == 1, f2 = t == 2, f3 = t == 3;
            const double tg = ((at(f0, f1, f2, f3) + at(e0 + f0, e1 + f1, e2 + f2, e3 + f3)) -
                               (at(-f0, -f1, -f2, -f3) + at(e0 - f0, e1 - f1, e2 - f2, e3 - f3))) *
                              (0.25 * inv_h);
            acc += tg * tg;
        }
        q[d] = acc;
    }
}

}  // namespace ss4
