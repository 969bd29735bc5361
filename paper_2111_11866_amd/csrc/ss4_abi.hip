// extern "C" entry points of libsubsurf4d.so: argument checks, workspace
// planning and dispatch to the launchers.  No C++ exception crosses this file.
#include <cmath>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <string>

#include "ss4_internal.hpp"

namespace ss4 {

namespace {
thread_local std::string g_error;
std::mutex g_timing_mu;
bool g_timing_on = false;
TimingTotals g_timing;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

void set_error(const std::string& msg) { g_error = msg; }

bool timing_enabled()
{
    std::lock_guard<std::mutex> g(g_timing_mu);
    return g_timing_on;
}

void timing_add(double ms, int64_t launches, int64_t updates)
{
    std::lock_guard<std::mutex> g(g_timing_mu);
    g_timing.sweep_ms += ms;
    g_timing.sweep_launches += launches;
    g_timing.voxel_updates += updates;
    g_timing.solves += 1;
}

int resident_grid(const void* kernel) { return resident_grid_bs(kernel, kBlock); }

int resident_grid_bs(const void* kernel, int block)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(mu);
    auto key = std::make_pair(dev, kernel);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, 0) != hipSuccess || per <= 0) per = 1;
    int64_t grid = (int64_t)per * cus;
    grid = grid / kXcd * kXcd;
    if (grid < kXcd) grid = kXcd;
    if (grid > kGridCap) grid = kGridCap;
    cache[key] = (int)grid;
    return (int)grid;
}

int hip_fail(hipError_t e, const char* what)
{
    g_error = std::string(what) + ": " + hipGetErrorString(e);
    return SUBSURF4D_EDEVICE;
}

bool plan_workspace(const int32_t n[4], int32_t n_centres, int32_t precision, WsPlan* P)
{
    for (int d = 0; d < 4; ++d)
        if (n[d] < 1 || n[d] > (1 << 20)) return false;
    const Layout L = make_layout(n);
    if (L.npad > ((int64_t)1 << 40)) return false;
    P->L = L;
    P->n_centres = n_centres;
    P->precision = precision;
    size_t off = 0;
    P->ctrl = off; off += align256(sizeof(Ctrl));
    const int64_t ncol = (int64_t)L.ntm * ((L.n2 + 3) >> 2) * L.n3;   // one-block-per-column sweeps
    P->max_grid = ncol + kXcd > kGridCap ? ncol + kXcd : kGridCap;
    P->part_a = off; off += align256(sizeof(double) * P->max_grid);
    P->part_b = off; off += align256(sizeof(double) * P->max_grid);
    P->balls = off; off += align256(sizeof(double) * 2 * (size_t)(n_centres > 0 ? n_centres : 1));
    P->big = off;

    size_t s = off;
    P->ured0 = s; s += align256(sizeof(double) * L.usplit);
    P->ured1 = s; s += align256(sizeof(double) * L.usplit);
    P->ublack = s; s += align256(sizeof(double) * L.usplit);
    P->coef = s; s += align256(sizeof(double) * 2 * L.cblk);     // coefficients + rhs, tiled
    if (precision == SUBSURF4D_MIXED) {
        const int64_t recs = 2 * L.nrow_int * L.ntm * kTileSlots;      // both colours
        P->coef16 = s; s += align256(16 * (size_t)recs);                 // 8 x BF16 per cell
        P->rf32 = s; s += align256(sizeof(float) * (size_t)recs);        // scaled FP32 residual
        P->dred = s; s += align256(sizeof(float) * L.usplit);            // FP32 correction, split
        P->dblack = s; s += align256(sizeof(float) * L.usplit);
    }
    P->step_bytes = s - off;

    size_t q = off;
    P->I0 = q; q += align256(sizeof(double) * L.nint);
    P->ITH = q; q += align256(sizeof(double) * L.nint);
    P->S0 = q; q += align256(sizeof(double) * L.nint);
    P->S1 = q; q += align256(sizeof(double) * L.nint);
    const int64_t ncq = L.nrow_int * L.half;                        // cells of one colour, split numbering
    P->HR = q; q += align256(sizeof(double) * 2 * ncq);
    P->HJ = q; q += align256(sizeof(double) * 2 * ncq);
    P->R = q; q += align256(sizeof(double) * ncq);
    P->prep_bytes = q - off;

    P->total = off + (P->step_bytes > P->prep_bytes ? P->step_bytes : P->prep_bytes);
    return true;
}

}  // namespace ss4

using namespace ss4;

static_assert(sizeof(subsurf4d_grid) == 24, "grid layout");
static_assert(sizeof(subsurf4d_centre) == 16, "centre layout");
static_assert(sizeof(subsurf4d_prepare_params) == 80, "prepare params layout");
static_assert(sizeof(subsurf4d_step_params) == 80, "step params layout");
static_assert(sizeof(subsurf4d_result) == 32, "result layout");
static_assert(sizeof(subsurf4d_batch_job) == 80, "batch job layout");
static_assert(sizeof(subsurf4d_batch_prepare_job) == 104, "batch prepare job layout");
static_assert(sizeof(subsurf4d_cell) == 24, "cell record layout");

namespace {

int fail(int code, const char* msg)
{
    set_error(msg);
    return code;
}

int check_grid(const subsurf4d_grid* g)
{
    if (!g) return fail(SUBSURF4D_EINVAL, "grid is NULL");
    for (int d = 0; d < 4; ++d)
        if (g->n[d] < 1 || g->n[d] > (1 << 20)) return fail(SUBSURF4D_ESHAPE, "grid size out of range");
    if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(SUBSURF4D_EINVAL, "h must be positive and finite");
    return 0;
}

int check_ws(const WsPlan& P, void* ws, size_t bytes, size_t need = 0)
{
    if (!ws) return fail(SUBSURF4D_EINVAL, "workspace is NULL");
    if (need == 0) need = P.total;
    if (bytes < need) return fail(SUBSURF4D_EWORKSPACE, "workspace too small (see subsurf4d_workspace_bytes)");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(SUBSURF4D_EINVAL, "workspace must be 256-byte aligned");
    return 0;
}

constexpr int32_t kMaxIterCap = 1 << 30;

int check_step_params(const subsurf4d_step_params* p)
{
    if (!p) return fail(SUBSURF4D_EINVAL, "params is NULL");
    if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return fail(SUBSURF4D_EINVAL, "eps must be positive");
    if (!(p->tau >= 0.0) || !std::isfinite(p->tau)) return fail(SUBSURF4D_EINVAL, "tau must be >= 0");
    if (!(p->omega > 0.0 && p->omega < 2.0)) return fail(SUBSURF4D_EINVAL, "omega must be in (0,2)");
    if (!(p->tol >= 0.0)) return fail(SUBSURF4D_EINVAL, "tol must be >= 0");
    // iteration counts stay far from INT_MAX, so pass counters (max_iter + 1) cannot overflow
    if (p->fixed_iters <= 0 && (p->max_iter < 1 || p->max_iter > kMaxIterCap))
        return fail(SUBSURF4D_EINVAL, "max_iter must be in [1, 2^30]");
    if (p->fixed_iters > kMaxIterCap) return fail(SUBSURF4D_EINVAL, "fixed_iters must be <= 2^30");
    if (p->check_every < 0) return fail(SUBSURF4D_EINVAL, "check_every must be >= 0");
    if (p->precision != SUBSURF4D_FP64 && p->precision != SUBSURF4D_MIXED)
        return fail(SUBSURF4D_EINVAL, "unknown precision");
    if (p->rescale && !(p->ball_r >= 0.0 && p->ball_r <= 1e6)) return fail(SUBSURF4D_EINVAL, "ball_r out of range");
    if (p->precision == SUBSURF4D_MIXED) {
        if (!(p->refine_tol > 0.0)) return fail(SUBSURF4D_EINVAL, "refine_tol must be > 0");
        if (p->inner_sweeps < 1 || p->inner_sweeps > 1024)
            return fail(SUBSURF4D_EINVAL, "inner_sweeps must be in [1, 1024]");
    }
    const int known = SUBSURF4D_FLAG_NO_GRAPH | SUBSURF4D_FLAG_SWEEP_FLAT | SUBSURF4D_FLAG_SWEEP_MARCH |
                      SUBSURF4D_FLAG_ASYNC | SUBSURF4D_FLAG_SHORT_LAST_PASS;
    if (p->flags & ~known) return fail(SUBSURF4D_EINVAL, "unknown flags");
    if ((p->flags & SUBSURF4D_FLAG_SWEEP_FLAT) && (p->flags & SUBSURF4D_FLAG_SWEEP_MARCH))
        return fail(SUBSURF4D_EINVAL, "at most one sweep shape flag");
    return 0;
}

}  // namespace

#define SS4_GUARD_BEGIN try {
#define SS4_GUARD_END                                                      \
    }                                                                      \
    catch (const std::exception& e) { return fail(SUBSURF4D_EDEVICE, e.what()); } \
    catch (...) { return fail(SUBSURF4D_EDEVICE, "unknown C++ exception"); }

extern "C" {

size_t subsurf4d_workspace_bytes(const subsurf4d_grid* grid, int32_t n_centres, int32_t precision)
{
    try {
        if (!grid || n_centres < 0) return 0;
        for (int d = 0; d < 4; ++d)
            if (grid->n[d] < 1 || grid->n[d] > (1 << 20)) return 0;
        WsPlan P;
        if (!plan_workspace(grid->n, n_centres, precision, &P)) return 0;
        return P.total;
    } catch (...) {
        return 0;
    }
}

size_t subsurf4d_prepare_workspace_bytes(const subsurf4d_grid* grid, int32_t n_centres)
{
    try {
        if (!grid || n_centres < 0) return 0;
        for (int d = 0; d < 4; ++d)
            if (grid->n[d] < 1 || grid->n[d] > (1 << 20)) return 0;
        WsPlan P;
        if (!plan_workspace(grid->n, n_centres, SUBSURF4D_FP64, &P)) return 0;
        return P.big + P.prep_bytes;
    } catch (...) {
        return 0;
    }
}

namespace {

int check_prepare_params(const subsurf4d_prepare_params* params)
{
    if (!params) return fail(SUBSURF4D_EINVAL, "NULL argument");
    const subsurf4d_prepare_params& p = *params;
    if (!(p.K >= 0.0) || !std::isfinite(p.K)) return fail(SUBSURF4D_EINVAL, "K must be >= 0");
    if (!(p.delta >= 0.0) || !std::isfinite(p.delta) || !(p.vartheta >= 0.0) || !std::isfinite(p.vartheta))
        return fail(SUBSURF4D_EINVAL, "delta and vartheta must be finite and >= 0");
    if (!(p.lambda >= 0.0 && p.lambda <= 1.0)) return fail(SUBSURF4D_EINVAL, "lambda must be in [0,1]");
    if (!(p.ball_r >= 0.0 && p.ball_r <= 1e6)) return fail(SUBSURF4D_EINVAL, "ball_r out of range");
    if (!(p.smooth_tau >= 0.0) || !std::isfinite(p.smooth_tau) || p.smooth_steps < 0)
        return fail(SUBSURF4D_EINVAL, "bad smoothing parameters");
    if (p.smooth_steps > 0 && (!(p.smooth_omega < 2.0) || p.smooth_max_iter < 1 ||
                               p.smooth_max_iter > kMaxIterCap || !(p.smooth_tol >= 0.0)))
        return fail(SUBSURF4D_EINVAL, "bad smoothing solver parameters");
    if (!std::isfinite(p.image_scale)) return fail(SUBSURF4D_EINVAL, "image_scale must be finite");
    return 0;
}

}  // namespace

int subsurf4d_prepare_g(const subsurf4d_grid* grid, const void* image, int32_t image_dtype,
                        const subsurf4d_centre* centres, int32_t n_centres,
                        const subsurf4d_prepare_params* params, double* G, int32_t* owner, void* workspace,
                        size_t workspace_bytes, void* stream)
{
    SS4_GUARD_BEGIN
    g_error.clear();
    if (int rc = check_grid(grid)) return rc;
    if (!image || !params || !G || !owner) return fail(SUBSURF4D_EINVAL, "NULL argument");
    if (n_centres < 0 || (n_centres > 0 && !centres)) return fail(SUBSURF4D_EINVAL, "bad centres");
    if (image_dtype != SUBSURF4D_U8 && image_dtype != SUBSURF4D_F32 && image_dtype != SUBSURF4D_F64)
        return fail(SUBSURF4D_EINVAL, "unknown image dtype");
    if (int rc = check_prepare_params(params)) return rc;
    const subsurf4d_prepare_params& p = *params;
    WsPlan P;
    if (!plan_workspace(grid->n, n_centres, SUBSURF4D_FP64, &P)) return fail(SUBSURF4D_ESHAPE, "grid too large");
    if (int rc = check_ws(P, workspace, workspace_bytes, P.big + P.prep_bytes)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int rc = run_prepare(P, grid->h, image, image_dtype, centres, n_centres, p, G, owner, workspace, s);
    if (rc < 0) return rc;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "prepare");
    return rc;
    SS4_GUARD_END
}

int subsurf4d_init_u(const subsurf4d_grid* grid, const subsurf4d_centre* seeds, int32_t n_seeds, double v,
                     double R, double* u, void* stream)
{
    SS4_GUARD_BEGIN
    g_error.clear();
    if (int rc = check_grid(grid)) return rc;
    if (!u || n_seeds < 0 || (n_seeds > 0 && !seeds)) return fail(SUBSURF4D_EINVAL, "bad arguments");
    if (!(v > 0.0) || !std::isfinite(v)) return fail(SUBSURF4D_EINVAL, "v must be positive");
    if (!std::isfinite(R) || R > 1e6) return fail(SUBSURF4D_EINVAL, "R out of range");
    const Layout L = make_layout(grid->n);
    return run_init_u(L, seeds, n_seeds, v, R, u, static_cast<hipStream_t>(stream));
    SS4_GUARD_END
}

int subsurf4d_rescale(const subsurf4d_grid* grid, const subsurf4d_centre* centres, int32_t n_centres,
                      double ball_r, const int32_t* owner, double* u, void* workspace, size_t workspace_bytes,
                      void* stream)
{
    SS4_GUARD_BEGIN
    g_error.clear();
    if (int rc = check_grid(grid)) return rc;
    if (!u || !owner || n_centres < 0 || (n_centres > 0 && !centres)) return fail(SUBSURF4D_EINVAL, "bad arguments");
    if (!(ball_r >= 0.0 && ball_r <= 1e6)) return fail(SUBSURF4D_EINVAL, "ball_r out of range");
    WsPlan P;
    if (!plan_workspace(grid->n, n_centres, SUBSURF4D_FP64, &P)) return fail(SUBSURF4D_ESHAPE, "grid too large");
    if (int rc = check_ws(P, workspace, workspace_bytes, P.big)) return rc;
    return run_rescale(P, centres, n_centres, ball_r, owner, u, workspace, static_cast<hipStream_t>(stream));
    SS4_GUARD_END
}

int subsurf4d_assemble(const subsurf4d_grid* grid, const double* G, const double* u,
                       const subsurf4d_step_params* params, double* coef, double* b, void* stream)
{
    SS4_GUARD_BEGIN
    g_error.clear();
    if (int rc = check_grid(grid)) return rc;
    if (!G || !u || !coef || !b) return fail(SUBSURF4D_EINVAL, "NULL argument");
    if (int rc = check_step_params(params)) return rc;
    const Layout L = make_layout(grid->n);
    return run_assemble_export(L, grid->h, G, u, *params, coef, b, static_cast<hipStream_t>(stream));
    SS4_GUARD_END
}

namespace {

int step_common(const subsurf4d_grid* grid, const double* G, const double* ub, const subsurf4d_centre* centres,
                int32_t n_centres, const int32_t* owner, double* u, const subsurf4d_step_params* params,
                subsurf4d_result* result, void* workspace, size_t workspace_bytes, void* stream)
{
    if (int rc = check_grid(grid)) return rc;
    if (!G || !u) return fail(SUBSURF4D_EINVAL, "NULL argument");
    if (int rc = check_step_params(params)) return rc;
    if (params->rescale && (n_centres < 0 || (n_centres > 0 && (!centres || !owner))))
        return fail(SUBSURF4D_EINVAL, "rescale needs centres and owner");
    const int nc = params->rescale ? n_centres : 0;
    WsPlan P;
    if (!plan_workspace(grid->n, nc, params->precision, &P)) return fail(SUBSURF4D_ESHAPE, "grid too large");
    if (int rc = check_ws(P, workspace, workspace_bytes)) return rc;
    // enqueue-only calls write the outcome on the device, into `result` if given
    subsurf4d_result tmp;
    const bool async = (params->flags & SUBSURF4D_FLAG_ASYNC) != 0;
    return run_step(P, grid->h, G, ub, centres, nc, owner, u, *params, result || async ? result : &tmp, workspace,
                    static_cast<hipStream_t>(stream));
}

}  // namespace

int subsurf4d_step(const subsurf4d_grid* grid, const double* G, const subsurf4d_centre* centres,
                   int32_t n_centres, const int32_t* owner, double* u, const subsurf4d_step_params* params,
                   subsurf4d_result* result, void* workspace, size_t workspace_bytes, void* stream)
{
    SS4_GUARD_BEGIN
    g_error.clear();
    return step_common(grid, G, nullptr, centres, n_centres, owner, u, params, result, workspace, workspace_bytes,
                       stream);
    SS4_GUARD_END
}

}  // extern "C"

namespace {

// Device scratch of subsurf4d_step_noalloc: one fixed array in each device's
// copy of the code object, in place of a caller workspace.  Host code never
// passes `scratch` itself to a kernel (on the host it names a stand-in, not a
// device address): the device address of each device's copy is looked up
// once per device, with that device current, and kept.
static __device__ __align__(256) unsigned char scratch[SUBSURF4D_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;

int scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "step_noalloc: current device");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "step_noalloc: address of the device scratch");
        if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0)
            return fail(SUBSURF4D_EDEVICE, "step_noalloc: device scratch is not 256-byte aligned");
        it = g_scratch_ptr.emplace(dev, p).first;
    }
    *out = it->second;
    return 0;
}

}  // namespace

extern "C" {

int subsurf4d_step_noalloc(const subsurf4d_grid* grid, const double* G, const subsurf4d_centre* centres,
                           int32_t n_centres, const int32_t* owner, double* u,
                           const subsurf4d_step_params* params, subsurf4d_result* result, void* stream)
{
    SS4_GUARD_BEGIN
    g_error.clear();
    if (int rc = check_grid(grid)) return rc;
    if (int rc = check_step_params(params)) return rc;
    const int nc = params->rescale ? n_centres : 0;
    WsPlan P;
    if (nc < 0 || !plan_workspace(grid->n, nc, params->precision, &P))
        return fail(SUBSURF4D_ESHAPE, "grid too large");
    if (P.total > (size_t)SUBSURF4D_NOALLOC_SCRATCH_BYTES)
        return fail(SUBSURF4D_EWORKSPACE, "step_noalloc: the grid needs more workspace than the library's "
                                          "fixed device scratch (SUBSURF4D_NOALLOC_SCRATCH_BYTES); use "
                                          "subsurf4d_step with a caller workspace");
    void* ws = nullptr;
    if (int rc = scratch_address(&ws)) return rc;
    return step_common(grid, G, nullptr, centres, n_centres, owner, u, params, result, ws,
                       (size_t)SUBSURF4D_NOALLOC_SCRATCH_BYTES, stream);
    SS4_GUARD_END
}

int subsurf4d_step_dirichlet(const subsurf4d_grid* grid, const double* G, const double* u_dirichlet,
                             const subsurf4d_centre* centres, int32_t n_centres, const int32_t* owner, double* u,
                             const subsurf4d_step_params* params, subsurf4d_result* result, void* workspace,
                             size_t workspace_bytes, void* stream)
{
    SS4_GUARD_BEGIN
    g_error.clear();
    if (!u_dirichlet) return fail(SUBSURF4D_EINVAL, "NULL Dirichlet data");
    if (u_dirichlet == u) return fail(SUBSURF4D_EINVAL, "Dirichlet data must be a separate array (or use subsurf4d_step)");
    return step_common(grid, G, u_dirichlet, centres, n_centres, owner, u, params, result, workspace,
                       workspace_bytes, stream);
    SS4_GUARD_END
}

int subsurf4d_solve(const subsurf4d_grid* grid, const double* coef, const double* b, double* u,
                    const subsurf4d_step_params* params, subsurf4d_result* result, void* workspace,
                    size_t workspace_bytes, void* stream)
{
    SS4_GUARD_BEGIN
    g_error.clear();
    if (int rc = check_grid(grid)) return rc;
    if (!coef || !b || !u) return fail(SUBSURF4D_EINVAL, "NULL argument");
    if (int rc = check_step_params(params)) return rc;
    if (params->precision != SUBSURF4D_FP64) return fail(SUBSURF4D_EINVAL, "solve supports FP64 only");
    WsPlan P;
    if (!plan_workspace(grid->n, 0, SUBSURF4D_FP64, &P)) return fail(SUBSURF4D_ESHAPE, "grid too large");
    if (int rc = check_ws(P, workspace, workspace_bytes)) return rc;
    subsurf4d_result tmp;
    const bool async = (params->flags & SUBSURF4D_FLAG_ASYNC) != 0;
    return run_solve(P, coef, b, u, *params, result || async ? result : &tmp, workspace,
                     static_cast<hipStream_t>(stream));
    SS4_GUARD_END
}

int subsurf4d_stream_probe(const void* src, void* dst, size_t bytes, int32_t reads, int32_t writes, int32_t reps,
                           double* ms, void* stream)
{
    SS4_GUARD_BEGIN
    g_error.clear();
    if (!src || !dst || !ms || reps < 1 || reads < 1 || reads > 16 || writes < 0 || writes > 1)
        return fail(SUBSURF4D_EINVAL, "bad arguments");
    if (bytes == 0 || bytes % 16 != 0) return fail(SUBSURF4D_EINVAL, "bytes must be a positive multiple of 16");
    if (reinterpret_cast<uintptr_t>(src) % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0)
        return fail(SUBSURF4D_EINVAL, "buffers must be 16-byte aligned");
    return run_stream_probe(src, dst, bytes, reads, writes, reps, ms, static_cast<hipStream_t>(stream));
    SS4_GUARD_END
}

int subsurf4d_copy_probe(const void* src, void* dst, size_t bytes, int32_t reps, double* ms, void* stream)
{
    SS4_GUARD_BEGIN
    g_error.clear();
    if (!src || !dst || !ms || reps < 1) return fail(SUBSURF4D_EINVAL, "bad arguments");
    if (bytes == 0 || bytes % 16 != 0) return fail(SUBSURF4D_EINVAL, "bytes must be a positive multiple of 16");
    if (reinterpret_cast<uintptr_t>(src) % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0)
        return fail(SUBSURF4D_EINVAL, "buffers must be 16-byte aligned");
    return run_copy_probe(src, dst, bytes, reps, ms, static_cast<hipStream_t>(stream));
    SS4_GUARD_END
}

size_t subsurf4d_batch_workspace_bytes(const subsurf4d_grid* grid, int32_t n_centres)
{
    try {
        if (!grid || n_centres < 0) return 0;
        return batch_job_bytes(grid->n, n_centres);
    } catch (...) {
        return 0;
    }
}

size_t subsurf4d_batch_table_bytes(int32_t n_jobs)
{
    return n_jobs > 0 ? batch_table_bytes(n_jobs) : 0;
}

int subsurf4d_step_batched(const subsurf4d_batch_job* jobs, int32_t n_jobs, const subsurf4d_step_params* params,
                           subsurf4d_result* results, void* table, size_t table_bytes, void* stream)
{
    SS4_GUARD_BEGIN
    g_error.clear();
    if (int rc = check_step_params(params)) return rc;
    if (n_jobs == 0) return SUBSURF4D_OK;
    if (!jobs || n_jobs < 0 || !table) return fail(SUBSURF4D_EINVAL, "bad batch arguments");
    if (params->flags & SUBSURF4D_FLAG_ASYNC)
        return fail(SUBSURF4D_EINVAL, "the batched step synchronises (no SUBSURF4D_FLAG_ASYNC)");
    if (params->inner_sweeps < 1 || params->inner_sweeps > 1024)
        return fail(SUBSURF4D_EINVAL, "inner_sweeps must be in [1, 1024]");
    if (reinterpret_cast<uintptr_t>(table) % 256 != 0) return fail(SUBSURF4D_EINVAL, "table must be 256-byte aligned");
    for (int q = 0; q < n_jobs; ++q) {
        const subsurf4d_batch_job& j = jobs[q];
        if (int rc = check_grid(&j.grid)) return rc;
        if (!j.G || !j.u || !j.workspace) return fail(SUBSURF4D_EINVAL, "batch job with a NULL pointer");
        if (reinterpret_cast<uintptr_t>(j.workspace) % 256 != 0)
            return fail(SUBSURF4D_EINVAL, "job workspace must be 256-byte aligned");
        if (params->rescale && (j.n_centres < 0 || (j.n_centres > 0 && (!j.centres || !j.owner))))
            return fail(SUBSURF4D_EINVAL, "rescale needs centres and owner");
    }
    return run_batch_step(jobs, n_jobs, *params, results, table, table_bytes, static_cast<hipStream_t>(stream));
    SS4_GUARD_END
}

int subsurf4d_prepare_batched(const subsurf4d_batch_prepare_job* jobs, int32_t n_jobs,
                              const subsurf4d_prepare_params* params, double v, double R, double ball_r,
                              int32_t* statuses, void* table, size_t table_bytes, void* stream)
{
    SS4_GUARD_BEGIN
    g_error.clear();
    if (int rc = check_prepare_params(params)) return rc;
    if (n_jobs == 0) return SUBSURF4D_OK;
    if (!jobs || n_jobs < 0 || !table) return fail(SUBSURF4D_EINVAL, "bad batch arguments");
    if (!(v > 0.0) || !std::isfinite(v)) return fail(SUBSURF4D_EINVAL, "v must be positive");
    if (!std::isfinite(R) || R > 1e6) return fail(SUBSURF4D_EINVAL, "R out of range");
    if (!std::isfinite(ball_r) || ball_r > 1e6) return fail(SUBSURF4D_EINVAL, "ball_r out of range");
    if (reinterpret_cast<uintptr_t>(table) % 256 != 0) return fail(SUBSURF4D_EINVAL, "table must be 256-byte aligned");
    for (int q = 0; q < n_jobs; ++q) {
        const subsurf4d_batch_prepare_job& j = jobs[q];
        if (int rc = check_grid(&j.grid)) return rc;
        if (!j.image || !j.G || !j.owner || !j.u || !j.workspace)
            return fail(SUBSURF4D_EINVAL, "batch job with a NULL pointer");
        if (j.image_dtype != SUBSURF4D_U8 && j.image_dtype != SUBSURF4D_F32 && j.image_dtype != SUBSURF4D_F64)
            return fail(SUBSURF4D_EINVAL, "unknown image dtype");
        if (j.n_centres < 0 || (j.n_centres > 0 && !j.centres)) return fail(SUBSURF4D_EINVAL, "bad centres");
        if (j.n_seeds < 0 || (j.n_seeds > 0 && !j.seeds)) return fail(SUBSURF4D_EINVAL, "bad seeds");
        if (reinterpret_cast<uintptr_t>(j.workspace) % 256 != 0)
            return fail(SUBSURF4D_EINVAL, "job workspace must be 256-byte aligned");
    }
    return run_batch_prepare(jobs, n_jobs, *params, v, R, ball_r, statuses, table, table_bytes,
                             static_cast<hipStream_t>(stream));
    SS4_GUARD_END
}

size_t subsurf4d_track_workspace_bytes(const subsurf4d_grid* grid, int32_t capacity)
{
    try {
        if (!grid || capacity < 0) return 0;
        for (int d = 0; d < 4; ++d)
            if (grid->n[d] < 1 || grid->n[d] > (1 << 20)) return 0;
        const int64_t N = (int64_t)grid->n[0] * grid->n[1] * grid->n[2] * grid->n[3];
        if (N >= ((int64_t)1 << 31)) return 0;
        return track_workspace_bytes(grid->n, capacity);
    } catch (...) {
        return 0;
    }
}

int subsurf4d_track(const subsurf4d_grid* grid, const double* u, double level, int32_t* label, int32_t* dist2,
                    subsurf4d_cell* cells, int32_t capacity, int32_t* n_cells, void* workspace,
                    size_t workspace_bytes, void* stream)
{
    SS4_GUARD_BEGIN
    g_error.clear();
    if (int rc = check_grid(grid)) return rc;
    if (!u || !label || !dist2 || !n_cells || capacity < 0 || (capacity > 0 && !cells))
        return fail(SUBSURF4D_EINVAL, "NULL argument");
    if (!std::isfinite(level)) return fail(SUBSURF4D_EINVAL, "level must be finite");
    const int64_t N = (int64_t)grid->n[0] * grid->n[1] * grid->n[2] * grid->n[3];
    if (N >= ((int64_t)1 << 31)) return fail(SUBSURF4D_ESHAPE, "tracking names voxels by 32-bit indices");
    if (!workspace) return fail(SUBSURF4D_EINVAL, "workspace is NULL");
    if (workspace_bytes < track_workspace_bytes(grid->n, capacity))
        return fail(SUBSURF4D_EWORKSPACE, "workspace too small (see subsurf4d_track_workspace_bytes)");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(SUBSURF4D_EINVAL, "workspace must be 256-byte aligned");
    return run_track(grid->n, u, level, label, dist2, cells, capacity, n_cells, workspace,
                     static_cast<hipStream_t>(stream));
    SS4_GUARD_END
}

int subsurf4d_track_join(const subsurf4d_grid* grid, subsurf4d_cell* cells, int32_t n_cells, double radius)
{
    SS4_GUARD_BEGIN
    g_error.clear();
    if (int rc = check_grid(grid)) return rc;
    if (n_cells < 0 || (n_cells > 0 && !cells)) return fail(SUBSURF4D_EINVAL, "bad cells");
    if (!(radius >= 0.0) || !std::isfinite(radius)) return fail(SUBSURF4D_EINVAL, "radius must be >= 0");
    return run_track_join(grid->n, cells, n_cells, radius);
    SS4_GUARD_END
}

const char* subsurf4d_status_string(int status)
{
    switch (status) {
    case SUBSURF4D_OK: return "ok";
    case SUBSURF4D_NOT_CONVERGED: return "not converged (iteration cap reached)";
    case SUBSURF4D_EINVAL: return "invalid argument";
    case SUBSURF4D_ESHAPE: return "unsupported grid shape";
    case SUBSURF4D_EWORKSPACE: return "workspace too small";
    case SUBSURF4D_ENONFINITE: return "non-finite value";
    case SUBSURF4D_EDEVICE: return "HIP device error";
    default: return "unknown status";
    }
}

const char* subsurf4d_last_error(void) { return g_error.c_str(); }

const char* subsurf4d_version(void) { return "subsurf4d 0.1 (gfx950)"; }

void subsurf4d_timing(int32_t op, double* sweep_ms, int64_t* sweep_launches, int64_t* voxel_updates,
                      int64_t* solves)
{
    std::lock_guard<std::mutex> g(g_timing_mu);
    if (op == 1 || op == 0) g_timing_on = (op == 1);
    if (op == 2) g_timing = TimingTotals();
    if (sweep_ms) *sweep_ms = g_timing.sweep_ms;
    if (sweep_launches) *sweep_launches = g_timing.sweep_launches;
    if (voxel_updates) *voxel_updates = g_timing.voxel_updates;
    if (solves) *solves = g_timing.solves;
}

}  // extern "C"
