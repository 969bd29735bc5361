// Shared definitions of the gfx950 SUBSURF-4D library: grid layouts, the
// device control block, deterministic block reductions and launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "subsurf4d.h"

namespace ss4 {

constexpr int kBlock = 256;     // threads per block (4 wave64s)
constexpr int kXcd = 8;         // MI355X: 8 XCDs, blocks are dealt round-robin
constexpr int kGridCap = 8192;  // persistent-style grid cap (multiple of kXcd)

// ---------------------------------------------------------------- layouts
//
// Natural arrays are x-fastest.  "padded" includes one ghost layer per side.
//
// Colour-split ("red-black compacted") layout used by the sweeps: a cell
// (i,j,k,l) with colour c = (i+j+k+l)&1 is stored in colour array c, row
// (j,k,l), slot m = (i-1)>>1.  In a row with p = (c+j+k+l)&1 the cells of
// colour c have i&1 == p, i.e. i = 2m + 2 - p.  The x-neighbours i-1 and i+1
// (other colour, same row) sit at slots m-p and m+1-p; the y/z/t neighbours
// sit at the same slot m of the neighbouring rows.  u arrays keep every
// padded row (ghost rows and the x-ghost slots m=-1 and m=N1>>1 hold the
// Dirichlet data) so a sweep never needs a boundary test; coefficient and
// right-hand-side arrays keep interior rows only.
struct Layout {
    int n1, n2, n3, n4;     // interior sizes
    int p1, p2, p3, p4;     // padded sizes
    int half;               // (n1+1)/2 = most cells of one colour in a row
    int xoff;               // u-split slot of m = 0 (>= 1 leaves room for m = -1)
    int rs;                 // u-split row stride (doubles)
    int rsc;                // coefficient / rhs row stride (values)
    int64_t nrow_pad;       // p2*p3*p4
    int64_t nrow_int;       // n2*n3*n4
    int64_t npad, nint;     // padded / interior cell counts
    int64_t usplit;         // elements of one colour buffer of u
    int64_t csplit;         // elements of one colour of one coefficient array (row layout)
    int ntm;                // coefficient tiles (kTileSlots slots) per row
    int64_t cblk;           // values of one colour in the tiled coefficient block
};

// Tiled coefficient block of one colour: for every interior row and 64-slot
// tile, 9 fields (the 8 face coefficients in face order -x,+x,-y,+y,-z,+z,-t,+t,
// then the right-hand side) of 128 slots each, contiguous.  A wave that
// updates one tile reads one 9 KB run instead of nine streams.
constexpr int kTileShift = 7;
constexpr int kTileSlots = 1 << kTileShift;   // 128 slots
constexpr int kTileFields = 9;
constexpr int kTileVals = kTileFields * kTileSlots;

inline Layout make_layout(const int32_t n[4])
{
    Layout L;
    L.n1 = n[0]; L.n2 = n[1]; L.n3 = n[2]; L.n4 = n[3];
    L.p1 = n[0] + 2; L.p2 = n[1] + 2; L.p3 = n[2] + 2; L.p4 = n[3] + 2;
    L.half = (n[0] + 1) / 2;
    const bool wide = L.half >= 64;
    L.xoff = wide ? 16 : 1;                      // 128-byte aligned interior for wide rows
    const int need = L.xoff + n[0] / 2 + 2;      // slots m = -1 .. N1>>1, +1 for pair loads
    const int align = wide ? 16 : 2;
    L.rs = (need + align - 1) / align * align;
    L.rsc = wide ? (L.half + 15) / 16 * 16 : L.half;
    L.nrow_pad = (int64_t)L.p2 * L.p3 * L.p4;
    L.nrow_int = (int64_t)n[1] * n[2] * n[3];
    L.npad = (int64_t)L.p1 * L.nrow_pad;
    L.nint = (int64_t)n[0] * L.nrow_int;
    L.usplit = L.nrow_pad * L.rs;
    L.csplit = L.nrow_int * L.rsc;
    L.ntm = (L.half + kTileSlots - 1) / kTileSlots;
    L.cblk = L.nrow_int * L.ntm * kTileVals;
    return L;
}

// Index of the 16-byte mixed-precision record (8 BF16 coefficients divided by
// the FP64 diagonal) of slot m in interior row r of colour `colour`; the FP32
// scaled residual of the same cell uses the same index into a float array.
__host__ __device__ __forceinline__ int64_t mrec(const Layout& L, int colour, int64_t r, int m)
{
    return (((int64_t)colour * L.nrow_int + r) * L.ntm + (m >> kTileShift)) * kTileSlots + (m & (kTileSlots - 1));
}

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint32_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// Index of field 0 of slot m in interior row r of colour `colour` in the tiled
// coefficient block; field f is at +f*kTileSlots.
__host__ __device__ __forceinline__ int64_t ctile(const Layout& L, int colour, int64_t r, int m)
{
    return (((int64_t)colour * L.nrow_int + r) * L.ntm + (m >> kTileShift)) * kTileVals + (m & (kTileSlots - 1));
}

// ------------------------------------------------------- device control block
//
// One per workspace.  Written by the last-arriving block of a kernel (fixed
// order reduction of per-block partial sums) and read by later kernels and by
// the host between launch chunks.
struct Ctrl {
    unsigned int arrive[4];  // arrival counters, reset by the last block
    int done;                // 1: solve finished (converged, capped or failed)
    int iterations;          // k of the returned iterate
    int status;              // SUBSURF4D_* outcome
    int final_red;           // red ping-pong buffer holding the returned iterate
    double bn;               // ||b||_2
    double rel_res;          // last tested ||r||_2 / ||b||_2
    double tol;              // stopping tolerance
    int max_iter;
    int outer;               // refinement passes (mixed precision)
    double aux[4];           // scratch scalars (mixed precision)
};

// ---------------------------------------------------------- reductions
//
// Fixed-order reductions: wave64 butterfly, then the 4 waves of a block in
// order, then the per-block partials in index order by the last block.  The
// result is bitwise reproducible for a given grid size.

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Sum over a 256-thread block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds4)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) lds4[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) t = ((lds4[0] + lds4[1]) + lds4[2]) + lds4[3];
    __syncthreads();
    return t;
}

// Returns true in every thread of the block that arrives last at `counter`
// (out of `nblocks`).  Partial results written before the call by thread 0 are
// visible to the last block after it returns.
__device__ __forceinline__ bool arrive_last(unsigned int* counter, unsigned int nblocks, int* lds_flag)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned int old = atomicAdd(counter, 1u);
        *lds_flag = (old == nblocks - 1) ? 1 : 0;
    }
    __syncthreads();
    const bool last = *lds_flag != 0;
    if (last) __threadfence();
    return last;
}

// Sum of part[0..n) in a fixed order, valid in thread 0 of the block.
__device__ __forceinline__ double sum_partials(const double* part, int n, double* lds4)
{
    double s = 0.0;
    for (int q = threadIdx.x; q < n; q += kBlock) s += part[q];
    return block_sum(s, lds4);
}

// Products and sums that the compiler may not contract into fused
// multiply-adds: decisions (ball membership, thresholds) must be taken on
// exactly the values the plain definition gives, each operation rounded.
__device__ __forceinline__ double dist2_exact(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
    return (xx + yy) + zz;
}

// lambda*alpha + (1-lambda)*beta with every operation rounded separately
__device__ __forceinline__ double threshold_exact(double lam, double alpha, double beta)
{
#pragma clang fp contract(off)
    const double a = lam * alpha;
    const double b = (1.0 - lam) * beta;
    return a + b;
}

// Deal the tiles [0, ntiles) to the blocks of a grid of size gridDim.x (a
// multiple of kXcd) so that the blocks resident on one XCD walk a contiguous
// range of tiles (better L2 reuse of neighbouring rows).
struct TileWalk {
    int64_t t, end, step;
    __device__ TileWalk(int64_t ntiles)
    {
        const int xcd = blockIdx.x % kXcd;
        const int slot = blockIdx.x / kXcd;
        const int slots = gridDim.x / kXcd;
        const int64_t chunk = (ntiles + kXcd - 1) / kXcd;
        const int64_t beg = (int64_t)xcd * chunk;
        end = beg + chunk < ntiles ? beg + chunk : ntiles;
        t = beg + slot;
        step = slots;
    }
};

// (Re)initialise the control block on the stream (a kernel rather than a
// memset so that the sequence can be captured in a graph).
static __global__ void k_ctrl_init(Ctrl* C, double tol, int max_iter)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int a = 0; a < 4; ++a) C->arrive[a] = 0;
        C->done = 0;
        C->iterations = 0;
        C->status = SUBSURF4D_OK;
        C->final_red = 0;
        C->bn = 0.0;
        C->rel_res = 0.0;
        C->tol = tol;
        C->max_iter = max_iter;
        C->outer = 0;
        for (int a = 0; a < 4; ++a) C->aux[a] = 0.0;
    }
}

inline int grid_for(int64_t work_items, int per_block = kBlock)
{
    int64_t g = (work_items + per_block - 1) / per_block;
    if (g < kXcd) g = kXcd;
    if (g > kGridCap) g = kGridCap;
    return (int)((g + kXcd - 1) / kXcd * kXcd);
}

}  // namespace ss4
