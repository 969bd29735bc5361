// Per-job preparation kernels: ball ownership, local thresholding,
// implicit zero-Neumann presmoothing, face edge detector G, initial function,
// local rescaling (Sec. 3.1 and Sec. 3.2.2 of the paper).
#include <climits>
#include <cstdlib>
#include <cmath>
#include <type_traits>

#include "ss4_internal.hpp"

namespace ss4 {
namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Bounding box of B(c, r) in 1-based interior indices with one voxel of slack;
// membership is decided by the exact squared distance.
struct Box {
    int lo[3], hi[3], w[3];
    int64_t count;
};

__device__ __forceinline__ Box ball_box(const Layout& L, const subsurf4d_centre& c, double r)
{
    Box b;
    const double cc[3] = {(double)c.x, (double)c.y, (double)c.z};
    const int n[3] = {L.n1, L.n2, L.n3};
    b.count = 1;
    for (int a = 0; a < 3; ++a) {
        b.lo[a] = clampi((int)floor(cc[a] - r), 1, n[a]);
        b.hi[a] = clampi((int)ceil(cc[a] + r) + 2, 1, n[a]);
        b.w[a] = b.hi[a] - b.lo[a] + 1;
        b.count *= b.w[a];
    }
    return b;
}

__device__ __forceinline__ void box_cell(const Box& b, int64_t q, int& i, int& j, int& k)
{
    i = b.lo[0] + (int)(q % b.w[0]);
    const int64_t q2 = q / b.w[0];
    j = b.lo[1] + (int)(q2 % b.w[1]);
    k = b.lo[2] + (int)(q2 / b.w[1]);
}

__device__ __forceinline__ double cell_dist2(const subsurf4d_centre& c, int i, int j, int k)
{
    return dist2_exact((double)(i - 1) - (double)c.x, (double)(j - 1) - (double)c.y,
                       (double)(k - 1) - (double)c.z);
}

__device__ __forceinline__ int64_t iidx(const Layout& L, int i, int j, int k, int l)
{
    return (((int64_t)(l - 1) * L.n3 + (k - 1)) * L.n2 + (j - 1)) * L.n1 + (i - 1);
}

__device__ __forceinline__ int64_t pidx(const Layout& L, int i, int j, int k, int l)
{
    return (((int64_t)l * L.p3 + k) * L.p2 + j) * L.p1 + i;
}

__device__ __forceinline__ bool frame_ok(const Layout& L, const subsurf4d_centre& c)
{
    return c.frame >= 0 && c.frame < L.n4;
}

// ------------------------------------------------------------ fills / casts

__global__ void k_fill_u64(uint64_t* a, int64_t n, uint64_t v)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        a[q] = v;
}

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        a[q] = v;
}

__global__ void k_fill_f64(double* a, int64_t n, double v)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        a[q] = v;
}

__global__ void k_copy_f64(const double* __restrict__ a, double* __restrict__ b, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        b[q] = a[q];
}

__global__ void k_image_to_f64(const void* img, int dtype, double scale, double* out, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        double v;
        if (dtype == SUBSURF4D_U8) v = (double)static_cast<const uint8_t*>(img)[q];
        else if (dtype == SUBSURF4D_F32) v = (double)static_cast<const float*>(img)[q];
        else v = static_cast<const double*>(img)[q];
        out[q] = __dmul_rn(scale, v);
    }
}

// ------------------------------------------------------------ ownership

// Pass 1: smallest squared distance to a containing centre, per cell.
__global__ void k_owner_pass1(Layout L, const subsurf4d_centre* cs, double r, uint64_t* key)
{
    const subsurf4d_centre c = cs[blockIdx.x];
    if (!frame_ok(L, c)) return;
    const Box b = ball_box(L, c, r);
    const double r2 = __dmul_rn(r, r);
    for (int64_t q = threadIdx.x; q < b.count; q += blockDim.x) {
        int i, j, k;
        box_cell(b, q, i, j, k);
        const double d2 = cell_dist2(c, i, j, k);
        if (d2 <= r2)
            atomicMin((unsigned long long*)&key[iidx(L, i, j, k, c.frame + 1)],
                      (unsigned long long)__double_as_longlong(d2));
    }
}

// Pass 2: among the centres at that distance, the lowest index owns the cell.
__global__ void k_owner_pass2(Layout L, const subsurf4d_centre* cs, double r, const uint64_t* key,
                              int32_t* owner)
{
    const int m = blockIdx.x;
    const subsurf4d_centre c = cs[m];
    if (!frame_ok(L, c)) return;
    const Box b = ball_box(L, c, r);
    const double r2 = __dmul_rn(r, r);
    for (int64_t q = threadIdx.x; q < b.count; q += blockDim.x) {
        int i, j, k;
        box_cell(b, q, i, j, k);
        const double d2 = cell_dist2(c, i, j, k);
        if (d2 <= r2) {
            const int64_t cell = iidx(L, i, j, k, c.frame + 1);
            if (key[cell] == (uint64_t)__double_as_longlong(d2)) atomicMin(&owner[cell], m);
        }
    }
}

__global__ void k_owner_fix(int32_t* owner, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        if (owner[q] == INT_MAX) owner[q] = -1;
}

// min / max of a field over each ball (one block per ball).
__global__ void k_ball_minmax(Layout L, const subsurf4d_centre* cs, double r, const double* f,
                              int padded, double* mn, double* mx)
{
    __shared__ double s_lo[4], s_hi[4];
    const int m = blockIdx.x;
    const subsurf4d_centre c = cs[m];
    double lo = INFINITY, hi = -INFINITY;
    if (frame_ok(L, c)) {
        const Box b = ball_box(L, c, r);
        const double r2 = __dmul_rn(r, r);
        for (int64_t q = threadIdx.x; q < b.count; q += blockDim.x) {
            int i, j, k;
            box_cell(b, q, i, j, k);
            if (cell_dist2(c, i, j, k) <= r2) {
                const double v = padded ? f[pidx(L, i, j, k, c.frame + 1)] : f[iidx(L, i, j, k, c.frame + 1)];
                lo = fmin(lo, v);
                hi = fmax(hi, v);
            }
        }
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    if ((threadIdx.x & 63) == 0) { s_lo[threadIdx.x >> 6] = lo; s_hi[threadIdx.x >> 6] = hi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        mn[m] = fmin(fmin(s_lo[0], s_lo[1]), fmin(s_lo[2], s_lo[3]));
        mx[m] = fmax(fmax(s_hi[0], s_hi[1]), fmax(s_hi[2], s_hi[3]));
    }
}

// Local thresholding (Sec. 3.1): beta where I0 >= TH, alpha otherwise, on owned cells.
__global__ void k_threshold(int64_t n, const double* I0, const int32_t* owner, const double* alpha,
                            const double* beta, double lam, double* ITH)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int m = owner[q];
        if (m < 0) { ITH[q] = I0[q]; continue; }
        const double a = alpha[m], b = beta[m];
        const double th = threshold_exact(lam, a, b);
        ITH[q] = (I0[q] >= th) ? b : a;
    }
}

// Local rescaling map on owned cells (one block per ball; each cell has one owner).
__global__ void k_ball_map(Layout L, const subsurf4d_centre* cs, double r, const int32_t* owner,
                           const double* mu, const double* xi, double* u)
{
    const int m = blockIdx.x;
    const subsurf4d_centre c = cs[m];
    if (!frame_ok(L, c)) return;
    const double lo = mu[m], span = __dsub_rn(xi[m], lo);
    if (!(span >= 1e-12)) return;
    const Box b = ball_box(L, c, r);
    const double r2 = __dmul_rn(r, r);
    for (int64_t q = threadIdx.x; q < b.count; q += blockDim.x) {
        int i, j, k;
        box_cell(b, q, i, j, k);
        if (cell_dist2(c, i, j, k) <= r2 && owner[iidx(L, i, j, k, c.frame + 1)] == m) {
            const int64_t p = pidx(L, i, j, k, c.frame + 1);
            u[p] = __ddiv_rn(__dsub_rn(u[p], lo), span);
        }
    }
}

// ---------------------------------------------------- implicit heat step
//
// (1 + a n_P) J_P - a sum_{interior nbrs} J_nbr = rhs_P, a = tau_s/h^2, zero
// Neumann boundary (no flux through boundary faces), red-black SOR.

// Magic constants of the index divisions of the heat kernels: grids whose flat
// indices stay below 2^31 (NARROW) decode cells with 32-bit multiplies instead
// of 64-bit divisions, which bound these kernels by ALU work.
struct HeatDiv { uint64_t half, n1, n2, n3; };

// Cell (i, j, k, l) and interior index q of colour COLOR's flat index
// h = row*half + m (cell i = 2m + 2 - par of the row); false where the row has
// no such cell (a row of odd length holds one cell more of one colour).
template <int COLOR, bool NARROW>
__device__ __forceinline__ bool heat_cell(const Layout& L, const HeatDiv& M, int64_t h, int64_t& q, int& i, int& j,
                                          int& k, int& l)
{
    int64_t row;
    int m;
    if (NARROW) {
        const uint32_t hh = (uint32_t)h;
        const uint32_t r = fdiv(hh, M.half);
        m = (int)(hh - r * (uint32_t)L.half);
        const uint32_t r2 = fdiv(r, M.n2);
        j = (int)(r - r2 * (uint32_t)L.n2) + 1;
        const uint32_t r3 = fdiv(r2, M.n3);
        k = (int)(r2 - r3 * (uint32_t)L.n3) + 1;
        l = (int)r3 + 1;
        row = r;
    } else {
        row = h / L.half;
        m = (int)(h - row * L.half);
        j = (int)(row % L.n2) + 1;
        const int64_t r2 = row / L.n2;
        k = (int)(r2 % L.n3) + 1;
        l = (int)(r2 / L.n3) + 1;
    }
    const int par = (COLOR + j + k + l) & 1;
    if (m >= (par ? (L.n1 + 1) >> 1 : L.n1 >> 1)) return false;
    i = 2 * m + 2 - par;
    q = NARROW ? (int64_t)((uint32_t)row * (uint32_t)L.n1 + (uint32_t)(i - 1)) : row * L.n1 + (i - 1);
    return true;
}

// The heat solves run on colour-split copies: colour c's cells sit at
// c*ncq + h, h = row*half + m (cell i = 2m + 2 - par of interior row `row`).
// Within the other colour's half, a cell's x-neighbours are h - par and
// h + 1 - par, and its y-, z- and t-neighbours keep m in the adjacent row,
// plane and frame (h -+ half, half*N2, half*N2*N3), so every access of a
// sweep is a contiguous run.  Slots past a row's last cell of a colour hold 0
// and are never read.
template <int COLOR, bool NARROW>
__global__ __launch_bounds__(kBlock) void k_heat_split(Layout L, HeatDiv M, const double* __restrict__ nat,
                                                       double* __restrict__ out0, double* __restrict__ out1)
{
    const int64_t ncq = L.nrow_int * L.half;
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < ncq; h += (int64_t)gridDim.x * blockDim.x) {
        int64_t q;
        int i, j, k, l;
        const double v = heat_cell<COLOR, NARROW>(L, M, h, q, i, j, k, l) ? nat[q] : 0.0;
        out0[COLOR * ncq + h] = v;
        out1[COLOR * ncq + h] = v;
    }
}

template <int COLOR, bool NARROW>
__global__ __launch_bounds__(kBlock) void k_heat_merge(Layout L, HeatDiv M, const double* __restrict__ split,
                                                       double* __restrict__ nat)
{
    const int64_t ncq = L.nrow_int * L.half;
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < ncq; h += (int64_t)gridDim.x * blockDim.x) {
        int64_t q;
        int i, j, k, l;
        if (heat_cell<COLOR, NARROW>(L, M, h, q, i, j, k, l)) nat[q] = split[COLOR * ncq + h];
    }
}

// Half-sweep of colour COLOR in red-black pass p on the split copies, with the
// stopping rule's residual fused in.  The red sweep forms the red rows of
// iterate p-1, rhs - A J before their update (the black cells still hold
// iterate p-1), and keeps iterate p-1's red values in `saved`; the black sweep
// forms the black rows of iterate p right after their update (their red
// neighbours already hold iterate p).  Per-block partials: red rows in part_r,
// black rows in part_k.  The last block of the red sweep of pass p >= 2 judges
// iterate p-1; a system stopped there has its red cells put back by
// k_lhe_restore.
//
// A lane owns slot g = ((k-1)*N2 + (j-1))*half + m of every frame and marches
// through the frames (h = g + (l-1)*ncq2): the other colour's values at the
// lane's own slot in frames l-1, l and l+1 stay in registers, so each frame
// of the other colour is read once instead of three times.  The neighbours are
// summed in the order -x, +x, -y, +y, -z, +z, -t, +t.
template <int COLOR, bool NARROW>
__global__ __launch_bounds__(kBlock) void k_lhe_sweep(Layout L, HeatDiv M, double a, double omega,
                                                      const double* __restrict__ rhs, double* J,
                                                      double* __restrict__ saved, int p, double* part_r,
                                                      double* part_k, Ctrl* C)
{
    __shared__ double lds[4];
    __shared__ int flag;
    if (C->done) return;
    const int64_t ncq = L.nrow_int * L.half;
    const int64_t ncq2 = (int64_t)L.half * L.n2 * L.n3;   // slots of one frame
    const int64_t sy = L.half, sz = (int64_t)L.half * L.n2;
    const double* __restrict__ R = rhs + COLOR * ncq;
    const double* __restrict__ O = J + (1 - COLOR) * ncq;   // the other colour: read only
    double* __restrict__ W = J + COLOR * ncq;               // this colour: updated
    double acc = 0.0;
    // chunks of kBlock slots dealt XCD-contiguously, so the y and z
    // neighbour rows of a chunk are read by blocks of the same XCD (its L2)
    const int64_t nch = (ncq2 + kBlock - 1) / kBlock;
    for (TileWalk tw(nch); tw.t < tw.end; tw.t += tw.step) {
        const int64_t g = tw.t * kBlock + threadIdx.x;
        if (g >= ncq2) continue;
        int m, j, k;
        if (NARROW) {
            const uint32_t gg = (uint32_t)g;
            const uint32_t r = fdiv(gg, M.half);
            m = (int)(gg - r * (uint32_t)L.half);
            const uint32_t r2 = fdiv(r, M.n2);
            j = (int)(r - r2 * (uint32_t)L.n2) + 1;
            k = (int)r2 + 1;
        } else {
            const int64_t r = g / L.half;
            m = (int)(g - r * L.half);
            j = (int)(r % L.n2) + 1;
            k = (int)(r / L.n2) + 1;
        }
        double oprev = 0.0, ocur = O[g];
        for (int l = 1; l <= L.n4; ++l) {
            const int64_t h = g + (int64_t)(l - 1) * ncq2;
            const double onext = l < L.n4 ? O[h + ncq2] : 0.0;
            const int par = (COLOR + j + k + l) & 1;
            if (m < (par ? (L.n1 + 1) >> 1 : L.n1 >> 1)) {
                const int i = 2 * m + 2 - par;
                double s = R[h];
                int cnt = 0;
                // x-neighbours h - par and h + 1 - par: one of them is h itself
                if (i > 1) { s += a * (par ? O[h - 1] : ocur); ++cnt; }
                if (i < L.n1) { s += a * (par ? ocur : O[h + 1]); ++cnt; }
                if (j > 1) { s += a * O[h - sy]; ++cnt; }
                if (j < L.n2) { s += a * O[h + sy]; ++cnt; }
                if (k > 1) { s += a * O[h - sz]; ++cnt; }
                if (k < L.n3) { s += a * O[h + sz]; ++cnt; }
                if (l > 1) { s += a * oprev; ++cnt; }
                if (l < L.n4) { s += a * onext; ++cnt; }
                const double D = 1.0 + a * cnt;
                const double uold = W[h];
                const double unew = omega * (s / D) + (1.0 - omega) * uold;
                W[h] = unew;
                const double r = s - D * (COLOR == 0 ? uold : unew);
                acc += r * r;
                if (COLOR == 0) saved[h] = uold;
            }
            oprev = ocur;
            ocur = onext;
        }
    }
    const double bs = block_sum(acc, lds);
    if (threadIdx.x == 0) (COLOR == 0 ? part_r : part_k)[blockIdx.x] = bs;
    if (COLOR == 1 || p < 2) return;
    if (!arrive_last(&C->arrive[3], gridDim.x, &flag)) return;
    const double R2 = sum_partials(part_r, gridDim.x, lds) + sum_partials(part_k, gridDim.x, lds);
    if (threadIdx.x == 0) {
        const int it = p - 1;
        const double Rn = sqrt(R2);
        C->rel_res = C->bn > 0.0 ? Rn / C->bn : Rn;
        C->iterations = it;
        if (!(R2 < INFINITY)) { C->status = SUBSURF4D_ENONFINITE; C->done = 1; }
        else if (Rn <= C->tol * C->bn) C->done = 1;
        else if (it >= C->max_iter) { C->status = SUBSURF4D_NOT_CONVERGED; C->done = 1; }
        C->arrive[3] = 0;
    }
}

// A solve judged on iterate k >= 1 stopped in the red sweep of pass k+1, which
// had already moved its red cells on: put iterate k's red values back (red
// half of the split copy; the other slots are never read).
__global__ __launch_bounds__(kBlock) void k_lhe_restore(int64_t ncq, const double* __restrict__ saved,
                                                        double* __restrict__ J, const Ctrl* C)
{
    if (C->iterations < 1) return;
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < ncq; h += (int64_t)gridDim.x * blockDim.x)
        J[h] = saved[h];
}

// Residual ||rhs - A J||_2 (and ||rhs||_2 at k = 0); the last block applies the
// stopping rule of the heat solve.
template <bool NARROW>
__global__ __launch_bounds__(kBlock) void k_lhe_residual(Layout L, HeatDiv M, double a, const double* __restrict__ rhs,
                                                         const double* __restrict__ J, int k, double* part_r,
                                                         double* part_b, Ctrl* C)
{
    __shared__ double lds[4];
    __shared__ int flag;
    if (C->done) return;
    const int64_t sy = L.n1, sz = (int64_t)L.n1 * L.n2, st = sz * L.n3;
    double ar = 0.0, ab = 0.0;
    const int64_t nch = (L.nint + kBlock - 1) / kBlock;      // chunks dealt XCD-contiguously
    for (TileWalk tw(nch); tw.t < tw.end; tw.t += tw.step) {
        const int64_t q = tw.t * kBlock + threadIdx.x;
        if (q >= L.nint) continue;
        int i, j, kk, l;
        if (NARROW) {
            const uint32_t qq = (uint32_t)q;
            const uint32_t r = fdiv(qq, M.n1);
            i = (int)(qq - r * (uint32_t)L.n1) + 1;
            const uint32_t r2 = fdiv(r, M.n2);
            j = (int)(r - r2 * (uint32_t)L.n2) + 1;
            const uint32_t r3 = fdiv(r2, M.n3);
            kk = (int)(r2 - r3 * (uint32_t)L.n3) + 1;
            l = (int)r3 + 1;
        } else {
            i = (int)(q % L.n1) + 1;
            const int64_t row = q / L.n1;
            j = (int)(row % L.n2) + 1;
            const int64_t r2 = row / L.n2;
            kk = (int)(r2 % L.n3) + 1;
            l = (int)(r2 / L.n3) + 1;
        }
        double s = rhs[q];
        int cnt = 0;
        if (i > 1) { s += a * J[q - 1]; ++cnt; }
        if (i < L.n1) { s += a * J[q + 1]; ++cnt; }
        if (j > 1) { s += a * J[q - sy]; ++cnt; }
        if (j < L.n2) { s += a * J[q + sy]; ++cnt; }
        if (kk > 1) { s += a * J[q - sz]; ++cnt; }
        if (kk < L.n3) { s += a * J[q + sz]; ++cnt; }
        if (l > 1) { s += a * J[q - st]; ++cnt; }
        if (l < L.n4) { s += a * J[q + st]; ++cnt; }
        const double r = s - (1.0 + a * cnt) * J[q];
        ar += r * r;
        if (k == 0) ab += rhs[q] * rhs[q];
    }
    const double br = block_sum(ar, lds);
    const double bb = block_sum(ab, lds);
    if (threadIdx.x == 0) { part_r[blockIdx.x] = br; part_b[blockIdx.x] = bb; }
    if (!arrive_last(&C->arrive[3], gridDim.x, &flag)) return;
    const double R2 = sum_partials(part_r, gridDim.x, lds);
    const double B2 = k == 0 ? sum_partials(part_b, gridDim.x, lds) : 0.0;
    if (threadIdx.x == 0) {
        if (k == 0) C->bn = sqrt(B2);
        const double R = sqrt(R2);
        C->rel_res = C->bn > 0.0 ? R / C->bn : R;
        C->iterations = k;
        if (!(R2 < INFINITY)) { C->status = SUBSURF4D_ENONFINITE; C->done = 1; }
        else if (R <= C->tol * C->bn) C->done = 1;
        else if (k >= C->max_iter) { C->status = SUBSURF4D_NOT_CONVERGED; C->done = 1; }
        C->arrive[3] = 0;
    }
}

// --------------------------------------------------------- edge detector G

// G on the 4 "+" faces of every padded cell.  Both images are read through
// face_q4; NARROW grids (fewer than 2^31 padded cells) decode with 32-bit
// multiplies and index with 32-bit offsets.
template <bool NARROW>
__global__ __launch_bounds__(kBlock) void k_face_g(Layout L, uint64_t mp1, uint64_t mp2, uint64_t mp3, double inv_h,
                                                   double K, double delta, double vartheta,
                                                   const double* __restrict__ S0, const double* __restrict__ S1,
                                                   double* __restrict__ G)
{
    using IDX = typename std::conditional<NARROW, uint32_t, int64_t>::type;
    const int n[4] = {L.n1, L.n2, L.n3, L.n4};
    const IDX stride[4] = {1, (IDX)L.n1, (IDX)L.n1 * (IDX)L.n2, (IDX)L.n1 * (IDX)L.n2 * (IDX)L.n3};
    // chunks of kBlock cells dealt XCD-contiguously: the rows around a chunk
    // (y, z neighbours of both images) are read by blocks of the same XCD at
    // about the same time, so they come from its L2
    const int64_t nchunk = (L.npad + kBlock - 1) / kBlock;
    for (TileWalk tw(nchunk); tw.t < tw.end; tw.t += tw.step) {
        const int64_t p = tw.t * kBlock + threadIdx.x;
        if (p >= L.npad) continue;
        int c[4];
        if (NARROW) {
            const uint32_t pp = (uint32_t)p;
            const uint32_t row = fdiv(pp, mp1);
            c[0] = (int)(pp - row * (uint32_t)L.p1);
            const uint32_t r2 = fdiv(row, mp2);
            c[1] = (int)(row - r2 * (uint32_t)L.p2);
            const uint32_t r3 = fdiv(r2, mp3);
            c[2] = (int)(r2 - r3 * (uint32_t)L.p3);
            c[3] = (int)r3;
        } else {
            c[0] = (int)(p % L.p1);
            const int64_t row = p / L.p1;
            c[1] = (int)(row % L.p2);
            const int64_t r2 = row / L.p2;
            c[2] = (int)(r2 % L.p3);
            c[3] = (int)(r2 / L.p3);
        }
        IDX off[4][3];
#pragma unroll
        for (int d = 0; d < 4; ++d)
#pragma unroll
            for (int sh = -1; sh <= 1; ++sh) off[d][sh + 1] = (IDX)(clampi(c[d] + sh, 1, n[d]) - 1) * stride[d];
        double q0[4], q1[4];
        face_q4(S0, off, inv_h, q0);
        face_q4(S1, off, inv_h, q1);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const double s = delta * sqrt(q0[d]) + vartheta * sqrt(q1[d]);
            G[(int64_t)d * L.npad + p] = 1.0 / (1.0 + K * (s * s));
        }
    }
}

// ------------------------------------------------------- initial function

// R <= 0: every interior cell takes the max over its frame's seeds of 1/(|X-s|+v).
__global__ void k_init_u_dense(Layout L, const subsurf4d_centre* seeds, int ns, double v, double* u)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < L.npad; p += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(p % L.p1);
        const int64_t row = p / L.p1;
        const int j = (int)(row % L.p2);
        const int64_t r2 = row / L.p2;
        const int k = (int)(r2 % L.p3);
        const int l = (int)(r2 / L.p3);
        double best = 0.0;
        if (i >= 1 && i <= L.n1 && j >= 1 && j <= L.n2 && k >= 1 && k <= L.n3 && l >= 1 && l <= L.n4) {
            bool any = false;
            for (int m = 0; m < ns; ++m) {
                const subsurf4d_centre c = seeds[m];
                if (c.frame != l - 1) continue;
                const double val = __ddiv_rn(1.0, __dadd_rn(__dsqrt_rn(cell_dist2(c, i, j, k)), v));
                if (!any || val > best) best = val;
                any = true;
            }
        }
        u[p] = best;
    }
}

// R > 0: scatter max(0, 1/(|X-s|+v) - 1/(R+v)) over the seed's R-box (u starts at 0;
// non-negative doubles order like their bit patterns, so an integer max is exact).
__global__ void k_init_u_scatter(Layout L, const subsurf4d_centre* seeds, double v, double R, double* u)
{
    const subsurf4d_centre c = seeds[blockIdx.x];
    if (!frame_ok(L, c)) return;
    const Box b = ball_box(L, c, R);
    const double shift = __ddiv_rn(1.0, __dadd_rn(R, v));
    for (int64_t q = threadIdx.x; q < b.count; q += blockDim.x) {
        int i, j, k;
        box_cell(b, q, i, j, k);
        const double val = __dsub_rn(__ddiv_rn(1.0, __dadd_rn(__dsqrt_rn(cell_dist2(c, i, j, k)), v)), shift);
        if (val > 0.0)
            atomicMax((unsigned long long*)&u[pidx(L, i, j, k, c.frame + 1)],
                      (unsigned long long)__double_as_longlong(val));
    }
}

template <bool NARROW>
int lhe_solve_t(const WsPlan& P, double a, double omega, double tol, int max_iter, const double* rhs,
                double* J, void* ws, hipStream_t s, int* status)
{
    const Layout& L = P.L;
    Ctrl* C = ws_ptr<Ctrl>(ws, P.ctrl);
    double* pa = ws_ptr<double>(ws, P.part_a);
    double* pb = ws_ptr<double>(ws, P.part_b);
    double* saved = ws_ptr<double>(ws, P.R);
    double* HR = ws_ptr<double>(ws, P.HR);       // split right-hand side
    double* HJ = ws_ptr<double>(ws, P.HJ);       // split iterate
    const int gs = grid_for(L.nrow_int * L.half);
    const int gm = grid_for((int64_t)L.half * L.n2 * L.n3);   // marching sweeps: one lane per slot of a frame
    // the residual's per-block partials fit the workspace's partial arrays
    // (at least kGridCap entries), so it takes a full grid as well
    const int gr = grid_for(L.nint);
    const HeatDiv M{fdiv_magic((uint32_t)L.half), fdiv_magic((uint32_t)L.n1), fdiv_magic((uint32_t)L.n2),
                    fdiv_magic((uint32_t)L.n3)};
    k_copy_f64<<<grid_for(L.nint), kBlock, 0, s>>>(rhs, J, L.nint);
    k_ctrl_init<<<1, 64, 0, s>>>(C, tol, max_iter);
    k_lhe_residual<NARROW><<<gr, kBlock, 0, s>>>(L, M, a, rhs, J, 0, pa, pb, C);
    k_heat_split<0, NARROW><<<gs, kBlock, 0, s>>>(L, M, rhs, HR, HJ);
    k_heat_split<1, NARROW><<<gs, kBlock, 0, s>>>(L, M, rhs, HR, HJ);
    SS4_LAUNCHED("lhe residual");
    Ctrl hc;
    int k = 1, chunk = 4;
    for (;;) {
        SS4_HIP(hipMemcpyAsync(&hc, C, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
        SS4_HIP(hipStreamSynchronize(s));
        if (hc.done) break;
        // iterate k is judged in pass k+1, so up to max_iter + 1 passes
        if (k > max_iter + 1) {
            set_error("internal: heat solve ended without a decision");
            return SUBSURF4D_EDEVICE;
        }
        for (int c = 0; c < chunk && k <= max_iter + 1; ++c, ++k) {
            k_lhe_sweep<0, NARROW><<<gm, kBlock, 0, s>>>(L, M, a, omega, HR, HJ, saved, k, pa, pb, C);
            k_lhe_sweep<1, NARROW><<<gm, kBlock, 0, s>>>(L, M, a, omega, HR, HJ, saved, k, pa, pb, C);
        }
        SS4_LAUNCHED("lhe sweeps");
        if (chunk < 32) chunk *= 2;
    }
    k_lhe_restore<<<gs, kBlock, 0, s>>>(L.nrow_int * L.half, saved, HJ, C);
    k_heat_merge<0, NARROW><<<gs, kBlock, 0, s>>>(L, M, HJ, J);
    k_heat_merge<1, NARROW><<<gs, kBlock, 0, s>>>(L, M, HJ, J);
    SS4_LAUNCHED("lhe restore / merge");
    if (hc.status == SUBSURF4D_ENONFINITE) {
        set_error("non-finite residual in the presmoothing solve");
        return SUBSURF4D_ENONFINITE;
    }
    if (hc.status == SUBSURF4D_NOT_CONVERGED) *status = SUBSURF4D_NOT_CONVERGED;
    return 0;
}

// Grids below 2^31 cells take the 32-bit index decode.  SUBSURF4D_WIDE_INDEX=1
// forces the 64-bit form (read at every call), so that tests can check on
// small grids that both forms give the same bits.
bool wide_index_forced()
{
    const char* e = getenv("SUBSURF4D_WIDE_INDEX");
    return e && e[0] == '1';
}

int lhe_solve(const WsPlan& P, double a, double omega, double tol, int max_iter, const double* rhs,
              double* J, void* ws, hipStream_t s, int* status)
{
    const Layout& L = P.L;
    const bool narrow = L.nrow_int * L.half < ((int64_t)1 << 31) && L.nint < ((int64_t)1 << 31) &&
                        !wide_index_forced();
    return narrow ? lhe_solve_t<true>(P, a, omega, tol, max_iter, rhs, J, ws, s, status)
                  : lhe_solve_t<false>(P, a, omega, tol, max_iter, rhs, J, ws, s, status);
}

}  // namespace

int run_prepare(const WsPlan& P, double h, const void* image, int dtype, const subsurf4d_centre* centres,
                int nc, const subsurf4d_prepare_params& pp, double* G, int32_t* owner, void* ws,
                hipStream_t s)
{
    const Layout& L = P.L;
    double* I0 = ws_ptr<double>(ws, P.I0);
    double* ITH = ws_ptr<double>(ws, P.ITH);
    double* S0 = ws_ptr<double>(ws, P.S0);
    double* S1 = ws_ptr<double>(ws, P.S1);
    uint64_t* key = ws_ptr<uint64_t>(ws, P.S0);  // dead before the smoothing starts
    double* alpha = ws_ptr<double>(ws, P.balls);
    double* beta = alpha + (nc > 0 ? nc : 1);
    const int gi = grid_for(L.nint);

    k_image_to_f64<<<gi, kBlock, 0, s>>>(image, dtype, pp.image_scale, I0, L.nint);
    k_fill_i32<<<gi, kBlock, 0, s>>>(owner, L.nint, INT_MAX);
    if (nc > 0) {
        k_fill_u64<<<gi, kBlock, 0, s>>>(key, L.nint, ~0ull);
        k_owner_pass1<<<nc, kBlock, 0, s>>>(L, centres, pp.ball_r, key);
        k_owner_pass2<<<nc, kBlock, 0, s>>>(L, centres, pp.ball_r, key, owner);
        k_ball_minmax<<<nc, kBlock, 0, s>>>(L, centres, pp.ball_r, I0, 0, alpha, beta);
    }
    k_owner_fix<<<gi, kBlock, 0, s>>>(owner, L.nint);
    k_threshold<<<gi, kBlock, 0, s>>>(L.nint, I0, owner, alpha, beta, pp.lambda, ITH);
    SS4_LAUNCHED("prepare: ownership / threshold");

    // presmoothing: ping-pong between the source buffer and S0 / S1
    int status = 0;
    double* src0 = I0;
    double* dst0 = S0;
    double* src1 = ITH;
    double* dst1 = S1;
    const double a = pp.smooth_tau / (h * h);
    // omega <= 0: Young's optimum for the interior Jacobi radius 2*dim*a/(1+2*dim*a)
    double omega = pp.smooth_omega;
    if (!(omega > 0.0)) {
        const double rho = 8.0 * a / (1.0 + 8.0 * a);
        omega = 2.0 / (1.0 + sqrt(1.0 - rho * rho));
    }
    for (int step = 0; step < pp.smooth_steps; ++step) {
        int rc = lhe_solve(P, a, omega, pp.smooth_tol, pp.smooth_max_iter, src0, dst0, ws, s, &status);
        if (rc) return rc;
        rc = lhe_solve(P, a, omega, pp.smooth_tol, pp.smooth_max_iter, src1, dst1, ws, s, &status);
        if (rc) return rc;
        double* t0 = src0; src0 = dst0; dst0 = t0;
        double* t1 = src1; src1 = dst1; dst1 = t1;
    }
    const uint64_t mp1 = fdiv_magic((uint32_t)L.p1), mp2 = fdiv_magic((uint32_t)L.p2), mp3 = fdiv_magic((uint32_t)L.p3);
    if (L.npad < ((int64_t)1 << 31) && !wide_index_forced())
        k_face_g<true><<<grid_for(L.npad), kBlock, 0, s>>>(L, mp1, mp2, mp3, 1.0 / h, pp.K, pp.delta, pp.vartheta,
                                                           src0, src1, G);
    else
        k_face_g<false><<<grid_for(L.npad), kBlock, 0, s>>>(L, mp1, mp2, mp3, 1.0 / h, pp.K, pp.delta, pp.vartheta,
                                                            src0, src1, G);
    SS4_LAUNCHED("prepare: face G");
    return status;
}

int run_init_u(const Layout& L, const subsurf4d_centre* seeds, int ns, double v, double R, double* u,
               hipStream_t s)
{
    if (R > 0.0) {
        k_fill_f64<<<grid_for(L.npad), kBlock, 0, s>>>(u, L.npad, 0.0);
        if (ns > 0) k_init_u_scatter<<<ns, kBlock, 0, s>>>(L, seeds, v, R, u);
    } else {
        k_init_u_dense<<<grid_for(L.npad), kBlock, 0, s>>>(L, seeds, ns, v, u);
    }
    SS4_LAUNCHED("init_u");
    return 0;
}

int run_rescale(const WsPlan& P, const subsurf4d_centre* centres, int nc, double r, const int32_t* owner,
                double* u, void* ws, hipStream_t s)
{
    if (nc <= 0) return 0;
    double* mu = ws_ptr<double>(ws, P.balls);
    double* xi = mu + nc;
    k_ball_minmax<<<nc, kBlock, 0, s>>>(P.L, centres, r, u, 1, mu, xi);
    k_ball_map<<<nc, kBlock, 0, s>>>(P.L, centres, r, owner, mu, xi, u);
    SS4_LAUNCHED("rescale");
    return 0;
}

}  // namespace ss4
