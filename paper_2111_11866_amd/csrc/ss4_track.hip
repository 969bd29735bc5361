// Cell tracking from the 4D segmentation (Sec. 5): cells of every frame as
// face-connected components of {u >= level}, the squared distance of every
// cell voxel to the nearest voxel outside its cell, each cell's centre (the
// voxel of largest distance), and the backward link of every cell to a cell
// of the previous frame; then, on the host, the joining of partial
// trajectories by tangent prolongation.
//
// Names: a cell is named by the smallest interior index of its voxels, so
// the output does not depend on the order in which threads visit voxels.
#include <algorithm>
#include <cstring>
#include <vector>

#include "ss4_internal.hpp"

namespace ss4 {
namespace {

struct TrackGeom {
    int n1, n2, n3, n4;
    int p1, p2, p3;
    int64_t fsz;          // voxels of one frame
    int64_t nint;         // interior voxels
};

__device__ __forceinline__ void decode(const TrackGeom& g, int64_t q, int& x, int& y, int& z, int& f)
{
    x = (int)(q % g.n1);
    int64_t r = q / g.n1;
    y = (int)(r % g.n2);
    r /= g.n2;
    z = (int)(r % g.n3);
    f = (int)(r / g.n3);
}

// label = own index where u >= level, -1 elsewhere
__global__ __launch_bounds__(kBlock) void kt_init(TrackGeom g, const double* __restrict__ u, double level, int32_t* lab)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < g.nint; q += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z, f;
        decode(g, q, x, y, z, f);
        const int64_t p = (((int64_t)(f + 1) * g.p3 + (z + 1)) * g.p2 + (y + 1)) * g.p1 + (x + 1);
        lab[q] = u[p] >= level ? (int32_t)q : -1;
    }
}

__device__ __forceinline__ int32_t find_root(int32_t* lab, int32_t a)
{
    int32_t b = __atomic_load_n(&lab[a], __ATOMIC_RELAXED);
    while (b != a) {
        a = b;
        b = __atomic_load_n(&lab[a], __ATOMIC_RELAXED);
    }
    return a;
}

// Union of v with its +x, +y, +z neighbours in the same frame: the larger
// root is hooked onto the smaller with atomicMin, retrying until both roots
// agree, so every component ends as one tree rooted at its smallest index.
__global__ __launch_bounds__(kBlock) void kt_union(TrackGeom g, int32_t* lab)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < g.nint; q += (int64_t)gridDim.x * blockDim.x) {
        if (lab[q] < 0) continue;
        int x, y, z, f;
        decode(g, q, x, y, z, f);
        const int64_t nb[3] = {x + 1 < g.n1 ? q + 1 : -1, y + 1 < g.n2 ? q + g.n1 : -1,
                               z + 1 < g.n3 ? q + (int64_t)g.n1 * g.n2 : -1};
        for (int s = 0; s < 3; ++s) {
            if (nb[s] < 0 || __atomic_load_n(&lab[nb[s]], __ATOMIC_RELAXED) < 0) continue;
            int32_t a = find_root(lab, (int32_t)q);
            int32_t b = find_root(lab, (int32_t)nb[s]);
            while (a != b) {
                if (a > b) { const int32_t t = a; a = b; b = t; }
                const int32_t old = atomicMin(&lab[b], a);
                if (old == b) break;            // b was a root and now hangs under a
                b = find_root(lab, old);
                a = find_root(lab, a);
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void kt_compress(TrackGeom g, int32_t* lab)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < g.nint; q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = lab[q];
        if (a >= 0) lab[q] = find_root(lab, a);
    }
}

// Exact squared Euclidean distance to the nearest voxel outside the cell (the
// outside of the image counts as outside), separably: along x the distance
// to the nearest voxel in no cell, then the lower envelope along y and along
// z, each scan stopping when the offset alone reaches the best value.  (A
// voxel of another cell is never nearer than the nearest voxel in no cell:
// a face path between two cells passes through a voxel in no cell.)
__global__ __launch_bounds__(kBlock) void kt_edt_x(TrackGeom g, const int32_t* __restrict__ lab, int32_t* out)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < g.nint; q += (int64_t)gridDim.x * blockDim.x) {
        if (lab[q] < 0) { out[q] = 0; continue; }
        const int x = (int)(q % g.n1);
        int dl = 1;
        while (x - dl >= 0 && lab[q - dl] >= 0) ++dl;
        int dr = 1;
        while (x + dr < g.n1 && lab[q + dr] >= 0) ++dr;
        const int d = dl < dr ? dl : dr;
        out[q] = d * d;
    }
}

// pass along axis with stride `st` and extent `ext` (coordinate c of q)
template <int AXIS>
__global__ __launch_bounds__(kBlock) void kt_edt_pass(TrackGeom g, const int32_t* __restrict__ lab,
                                                      const int32_t* __restrict__ in, int32_t* out)
{
    const int64_t st = AXIS == 1 ? (int64_t)g.n1 : (int64_t)g.n1 * g.n2;
    const int ext = AXIS == 1 ? g.n2 : g.n3;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < g.nint; q += (int64_t)gridDim.x * blockDim.x) {
        if (lab[q] < 0) { out[q] = 0; continue; }
        const int c = AXIS == 1 ? (int)((q / g.n1) % g.n2) : (int)((q / ((int64_t)g.n1 * g.n2)) % g.n3);
        int best = in[q];
        for (int s = 1; s * s < best; ++s) {
            const int s2 = s * s;
            // outside the image the value is 0
            const int lo = c - s >= 0 ? in[q - s * st] : 0;
            const int hi = c + s < ext ? in[q + s * st] : 0;
            const int m = lo < hi ? lo : hi;
            if (m + s2 < best) best = m + s2;
        }
        out[q] = best;
    }
}

// Roots (voxels naming their cell) counted per block of a fixed voxel range,
// then numbered in index order: rank_at[root] = rank.
constexpr int kRange = 4096;

__global__ __launch_bounds__(kBlock) void kt_count_roots(TrackGeom g, const int32_t* __restrict__ lab, int32_t* cnt)
{
    __shared__ int s[4];
    const int64_t beg = (int64_t)blockIdx.x * kRange;
    int c = 0;
    for (int64_t q = beg + threadIdx.x; q < beg + kRange && q < g.nint; q += kBlock) c += lab[q] == (int32_t)q;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

__global__ __launch_bounds__(kBlock) void kt_rank_roots(TrackGeom g, const int32_t* __restrict__ lab,
                                                        const int32_t* __restrict__ base, int32_t* rank_at,
                                                        int32_t* cell_name)
{
    __shared__ int s[4];
    const int64_t beg = (int64_t)blockIdx.x * kRange;
    int next = base[blockIdx.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t c0 = beg; c0 < beg + kRange && c0 < g.nint; c0 += kBlock) {
        const int64_t q = c0 + threadIdx.x;
        const bool root = q < g.nint && q < beg + kRange && lab[q] == (int32_t)q;
        const uint64_t m = __ballot(root);
        const int below = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) s[w] = __popcll(m);
        __syncthreads();
        int before = 0;
        for (int t = 0; t < w; ++t) before += s[t];
        if (root) {
            const int r = next + before + below;
            rank_at[q] = r;
            cell_name[r] = (int32_t)q;
        }
        next += s[0] + s[1] + s[2] + s[3];
        __syncthreads();
    }
}

// Centre of every cell: the largest d2, ties to the smallest index, as one
// atomicMax on (d2 << 32 | ~index).
__global__ __launch_bounds__(kBlock) void kt_centre(TrackGeom g, const int32_t* __restrict__ lab,
                                                    const int32_t* __restrict__ d2, const int32_t* __restrict__ rank_at,
                                                    unsigned long long* key)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < g.nint; q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = lab[q];
        if (a < 0) continue;
        const unsigned long long k =
            ((unsigned long long)(uint32_t)d2[q] << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)q);
        atomicMax(&key[rank_at[a]], k);
    }
}

__global__ void kt_zero_u64(unsigned long long* a, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) a[q] = 0ull;
}

__global__ void kt_zero_i32(int32_t* a, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) a[q] = 0;
}

// Link by the centre's voxel moved to the previous frame; cells whose centre
// lands outside every cell get miss_id >= 0 (numbered by an atomic counter and
// renumbered in name order on the host side of the call).
__global__ __launch_bounds__(kBlock) void kt_link(TrackGeom g, int32_t K, const int32_t* __restrict__ lab,
                                                  const int32_t* __restrict__ cell_name,
                                                  const unsigned long long* __restrict__ key, int32_t* prev,
                                                  int32_t* kind, int32_t* missed)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < K; c += (int64_t)gridDim.x * blockDim.x) {
        const int32_t name = cell_name[c];
        const int32_t centre = (int32_t)(0xFFFFFFFFu - (uint32_t)(key[c] & 0xFFFFFFFFull));
        const int64_t f = name / g.fsz;
        prev[c] = -1;
        kind[c] = 0;
        missed[c] = 0;
        if (f == 0) continue;
        const int32_t below = lab[centre - g.fsz];
        if (below >= 0) { prev[c] = below; kind[c] = 1; }
        else missed[c] = 1;
    }
}

// Overlap counts of the missed cells with rows [row0, row0 + rows): for every
// voxel of such a cell, the cell of the previous frame at the same place.
__global__ __launch_bounds__(kBlock) void kt_overlap(TrackGeom g, const int32_t* __restrict__ lab,
                                                     const int32_t* __restrict__ rank_at,
                                                     const int32_t* __restrict__ row_of, int32_t row0, int32_t rows,
                                                     int32_t K, int32_t* table)
{
    for (int64_t q = g.fsz + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < g.nint;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = lab[q];
        if (a < 0) continue;
        const int32_t row = row_of[rank_at[a]] - row0;
        if (row < 0 || row >= rows) continue;
        const int32_t b = lab[q - g.fsz];
        if (b < 0) continue;
        atomicAdd(&table[(int64_t)row * K + rank_at[b]], 1);
    }
}

// Largest overlap of every missed row, ties to the smallest rank (= name).
__global__ __launch_bounds__(kBlock) void kt_overlap_best(const int32_t* __restrict__ table, int32_t rows, int32_t K,
                                                          const int32_t* __restrict__ row_cell,
                                                          const int32_t* __restrict__ cell_name, int32_t row0,
                                                          int32_t* prev, int32_t* kind)
{
    __shared__ int s_cnt[kBlock];
    __shared__ int s_col[kBlock];
    for (int r = blockIdx.x; r < rows; r += gridDim.x) {
        int bc = 0, bcol = -1;
        for (int col = threadIdx.x; col < K; col += kBlock) {
            const int v = table[(int64_t)r * K + col];
            if (v > bc) { bc = v; bcol = col; }          // columns ascend per thread: first max kept
        }
        s_cnt[threadIdx.x] = bc;
        s_col[threadIdx.x] = bcol;
        __syncthreads();
        if (threadIdx.x == 0) {
            int best = 0, bestc = -1;
            for (int t = 0; t < kBlock; ++t) {
                const int v = s_cnt[t], c = s_col[t];
                if (v > best || (v == best && v > 0 && c < bestc)) { best = v; bestc = c; }
            }
            const int cell = row_cell[row0 + r];
            if (bestc >= 0) { prev[cell] = cell_name[bestc]; kind[cell] = 2; }
        }
        __syncthreads();
    }
}

}  // namespace

// Entries of the (missed cell x cell) overlap table: at least
// kTrackTableEntries and the capacity, and half the voxel count, so that on a
// volume one or two row chunks (each a pass over the labels) cover every
// missed cell.
static int64_t track_table_entries(int64_t nint, int32_t capacity)
{
    const int64_t t = capacity > kTrackTableEntries ? capacity : kTrackTableEntries;
    return t > nint / 2 ? t : nint / 2;
}

size_t track_workspace_bytes(const int32_t n[4], int32_t capacity)
{
    const int64_t N = (int64_t)n[0] * n[1] * n[2] * n[3];
    const int64_t blocks = (N + kRange - 1) / kRange;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t table = (size_t)track_table_entries(N, capacity);
    return al(4 * (size_t)N) * 2 + al(4 * (size_t)(blocks + 1)) * 2 + al(8 * (size_t)capacity) +
           al(4 * (size_t)capacity) * 6 + al(table * 4);
}

int run_track(const int32_t n[4], const double* u, double level, int32_t* lab, int32_t* d2, subsurf4d_cell* cells,
              int32_t capacity, int32_t* n_cells, void* ws, hipStream_t s)
{
    TrackGeom g;
    g.n1 = n[0]; g.n2 = n[1]; g.n3 = n[2]; g.n4 = n[3];
    g.p1 = n[0] + 2; g.p2 = n[1] + 2; g.p3 = n[2] + 2;
    g.fsz = (int64_t)n[0] * n[1] * n[2];
    g.nint = g.fsz * n[3];
    const int64_t blocks = (g.nint + kRange - 1) / kRange;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    char* w = static_cast<char*>(ws);
    int32_t* tmp = reinterpret_cast<int32_t*>(w); w += al(4 * (size_t)g.nint);
    int32_t* rank_at = reinterpret_cast<int32_t*>(w); w += al(4 * (size_t)g.nint);
    int32_t* cnt = reinterpret_cast<int32_t*>(w); w += al(4 * (size_t)(blocks + 1));
    int32_t* base = reinterpret_cast<int32_t*>(w); w += al(4 * (size_t)(blocks + 1));
    unsigned long long* key = reinterpret_cast<unsigned long long*>(w); w += al(8 * (size_t)capacity);
    int32_t* cell_name = reinterpret_cast<int32_t*>(w); w += al(4 * (size_t)capacity);
    int32_t* prev = reinterpret_cast<int32_t*>(w); w += al(4 * (size_t)capacity);
    int32_t* kind = reinterpret_cast<int32_t*>(w); w += al(4 * (size_t)capacity);
    int32_t* missed = reinterpret_cast<int32_t*>(w); w += al(4 * (size_t)capacity);
    int32_t* row_of = reinterpret_cast<int32_t*>(w); w += al(4 * (size_t)capacity);
    int32_t* row_cell = reinterpret_cast<int32_t*>(w); w += al(4 * (size_t)capacity);
    int32_t* table = reinterpret_cast<int32_t*>(w);

    const int grid = grid_for(g.nint);
    kt_init<<<grid, kBlock, 0, s>>>(g, u, level, lab);
    kt_union<<<grid, kBlock, 0, s>>>(g, lab);
    kt_compress<<<grid, kBlock, 0, s>>>(g, lab);
    kt_edt_x<<<grid, kBlock, 0, s>>>(g, lab, d2);
    kt_edt_pass<1><<<grid, kBlock, 0, s>>>(g, lab, d2, tmp);
    kt_edt_pass<2><<<grid, kBlock, 0, s>>>(g, lab, tmp, d2);
    kt_count_roots<<<(unsigned)blocks, kBlock, 0, s>>>(g, lab, cnt);
    SS4_LAUNCHED("track: labels and distances");

    // number the cells: exclusive scan of the per-range root counts
    std::vector<int32_t> hc((size_t)blocks), hb((size_t)blocks + 1);
    SS4_HIP(hipMemcpyAsync(hc.data(), cnt, 4 * (size_t)blocks, hipMemcpyDeviceToHost, s));
    SS4_HIP(hipStreamSynchronize(s));
    int64_t K = 0;
    for (int64_t b = 0; b < blocks; ++b) { hb[(size_t)b] = (int32_t)K; K += hc[(size_t)b]; }
    if (K > capacity) {
        *n_cells = (int32_t)(K < INT32_MAX ? K : INT32_MAX);
        set_error("track: more cells than the capacity (n_cells holds the count)");
        return SUBSURF4D_EWORKSPACE;
    }
    *n_cells = (int32_t)K;
    if (K == 0) return 0;
    SS4_HIP(hipMemcpyAsync(base, hb.data(), 4 * (size_t)blocks, hipMemcpyHostToDevice, s));
    kt_rank_roots<<<(unsigned)blocks, kBlock, 0, s>>>(g, lab, base, rank_at, cell_name);
    kt_zero_u64<<<grid_for(K), kBlock, 0, s>>>(key, K);
    kt_centre<<<grid, kBlock, 0, s>>>(g, lab, d2, rank_at, key);
    kt_link<<<grid_for(K), kBlock, 0, s>>>(g, (int32_t)K, lab, cell_name, key, prev, kind, missed);
    SS4_LAUNCHED("track: cells and centre links");

    // cells whose centre misses the previous frame: overlap counts in row
    // chunks of the dense (missed cell x cell) table
    std::vector<int32_t> hmiss((size_t)K);
    SS4_HIP(hipMemcpyAsync(hmiss.data(), missed, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
    SS4_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> hrow((size_t)K, -1), hrcell;
    for (int64_t c = 0; c < K; ++c)
        if (hmiss[(size_t)c]) { hrow[(size_t)c] = (int32_t)hrcell.size(); hrcell.push_back((int32_t)c); }
    const int32_t M = (int32_t)hrcell.size();
    if (M > 0) {
        SS4_HIP(hipMemcpyAsync(row_of, hrow.data(), 4 * (size_t)K, hipMemcpyHostToDevice, s));
        SS4_HIP(hipMemcpyAsync(row_cell, hrcell.data(), 4 * (size_t)M, hipMemcpyHostToDevice, s));
        // SUBSURF4D_TRACK_TABLE=<entries> caps the table (more, smaller row
        // chunks; the same records)
        int64_t tab = track_table_entries(g.nint, capacity);
        const char* ev = getenv("SUBSURF4D_TRACK_TABLE");
        if (ev) {
            const long long v = atoll(ev);
            if (v > 0 && v < tab) tab = v;
        }
        const int32_t rows = (int32_t)std::max<int64_t>(1, std::min<int64_t>(M, tab / K));
        for (int32_t r0 = 0; r0 < M; r0 += rows) {
            const int32_t nr = std::min(rows, M - r0);
            kt_zero_i32<<<grid_for((int64_t)nr * K), kBlock, 0, s>>>(table, (int64_t)nr * K);
            kt_overlap<<<grid, kBlock, 0, s>>>(g, lab, rank_at, row_of, r0, nr, (int32_t)K, table);
            kt_overlap_best<<<std::min(nr, 4096), kBlock, 0, s>>>(table, nr, (int32_t)K, row_cell, cell_name, r0, prev,
                                                                 kind);
        }
        SS4_LAUNCHED("track: overlaps");
    }
    std::vector<int32_t> hname((size_t)K), hprev((size_t)K), hkind((size_t)K);
    std::vector<unsigned long long> hkey((size_t)K);
    SS4_HIP(hipMemcpyAsync(hname.data(), cell_name, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
    SS4_HIP(hipMemcpyAsync(hprev.data(), prev, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
    SS4_HIP(hipMemcpyAsync(hkind.data(), kind, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
    SS4_HIP(hipMemcpyAsync(hkey.data(), key, 8 * (size_t)K, hipMemcpyDeviceToHost, s));
    SS4_HIP(hipStreamSynchronize(s));
    for (int64_t c = 0; c < K; ++c) {
        subsurf4d_cell& o = cells[c];
        o.name = hname[(size_t)c];
        o.frame = (int32_t)(hname[(size_t)c] / g.fsz);
        o.centre = (int32_t)(0xFFFFFFFFu - (uint32_t)(hkey[(size_t)c] & 0xFFFFFFFFull));
        o.dist2 = (int32_t)(hkey[(size_t)c] >> 32);
        o.prev = hprev[(size_t)c];
        o.kind = hkind[(size_t)c];
    }
    return 0;
}

// Joining of partial trajectories (Sec. 5, last step), on the host.  A cell
// that no cell of the next frame links to ends a partial trajectory, which
// runs back along the links to a cell without one.  A partial trajectory T
// whose first cell lies in frame f > 0 is joined after the partial
// trajectory S ending in frame f-1 when T's first point moved back by its
// first displacement (or kept, for a single cell) lies within `radius` of S's
// last point, or S's last point moved on by its last displacement lies within
// `radius` of T's first point; T takes the nearest such S (squared distance,
// ties to the smaller name of S's last cell), each S at most once, the T in
// the order of the names of their first cells.  A join sets the first cell's
// link to S's last cell with kind 3.
int run_track_join(const int32_t n[4], subsurf4d_cell* cells, int32_t nc, double radius)
{
    std::vector<int32_t> order((size_t)nc);
    for (int32_t c = 0; c < nc; ++c) order[(size_t)c] = c;
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cells[a].name < cells[b].name; });
    auto find = [&](int32_t name) -> int32_t {
        int32_t lo = 0, hi = nc - 1;
        while (lo <= hi) {
            const int32_t mid = (lo + hi) / 2;
            const int32_t v = cells[order[(size_t)mid]].name;
            if (v == name) return order[(size_t)mid];
            if (v < name) lo = mid + 1;
            else hi = mid - 1;
        }
        return -1;
    };
    std::vector<char> has_next((size_t)nc, 0);
    for (int32_t c = 0; c < nc; ++c) {
        if (cells[c].prev < 0) continue;
        const int32_t p = find(cells[c].prev);
        if (p < 0) {
            set_error("track join: a link names no cell of the list");
            return SUBSURF4D_EINVAL;
        }
        has_next[(size_t)p] = 1;
    }
    struct Partial { std::vector<int32_t> cells; };   // first frame -> last frame (cell positions)
    std::vector<Partial> parts;
    for (int32_t oi = 0; oi < nc; ++oi) {
        const int32_t c = order[(size_t)oi];
        if (has_next[(size_t)c]) continue;
        std::vector<int32_t> chain{c};
        while (cells[chain.back()].prev >= 0) chain.push_back(find(cells[chain.back()].prev));
        std::reverse(chain.begin(), chain.end());
        parts.push_back({chain});
    }
    const int64_t fsz = (int64_t)n[0] * n[1] * n[2];
    auto xyz = [&](int32_t c, int64_t v[3]) {
        const int64_t q = cells[c].centre % fsz;
        v[0] = q % n[0];
        v[1] = (q / n[0]) % n[1];
        v[2] = q / ((int64_t)n[0] * n[1]);
    };
    const double r2 = radius * radius;
    std::vector<char> used(parts.size(), 0);
    // candidates S by the frame of their last cell, with that cell's name, its
    // point and its forward prolongation (the choice below is a strict order
    // on (distance, name), so the order of the candidates does not matter)
    struct End { size_t s; int32_t name; int64_t e0[3], fwd[3]; };
    std::vector<std::vector<End>> ending((size_t)(n[3] > 0 ? n[3] : 1));
    for (size_t sidx = 0; sidx < parts.size(); ++sidx) {
        const int32_t last = parts[sidx].cells.back();
        End e;
        e.s = sidx;
        e.name = cells[last].name;
        xyz(last, e.e0);
        if (parts[sidx].cells.size() > 1) {
            int64_t e1[3];
            xyz(parts[sidx].cells[parts[sidx].cells.size() - 2], e1);
            for (int a = 0; a < 3; ++a) e.fwd[a] = 2 * e.e0[a] - e1[a];
        } else {
            for (int a = 0; a < 3; ++a) e.fwd[a] = e.e0[a];
        }
        const int32_t fl = cells[last].frame;
        if (fl >= 0 && fl < n[3]) ending[(size_t)fl].push_back(e);
    }
    std::vector<size_t> tord(parts.size());
    for (size_t t = 0; t < parts.size(); ++t) tord[t] = t;
    std::sort(tord.begin(), tord.end(),
              [&](size_t a, size_t b) { return cells[parts[a].cells[0]].name < cells[parts[b].cells[0]].name; });
    for (size_t t : tord) {
        const int32_t first = parts[t].cells[0];
        const int32_t f = cells[first].frame;
        if (f <= 0 || f > n[3]) continue;     // no frame before it (or a record outside the grid)
        int64_t c0[3], back[3];
        xyz(first, c0);
        if (parts[t].cells.size() > 1) {
            int64_t c1[3];
            xyz(parts[t].cells[1], c1);
            for (int a = 0; a < 3; ++a) back[a] = 2 * c0[a] - c1[a];
        } else {
            for (int a = 0; a < 3; ++a) back[a] = c0[a];
        }
        int64_t best_d = -1;
        int32_t best_last = -1;
        size_t best_s = 0;
        for (const End& e : ending[(size_t)(f - 1)]) {
            if (used[e.s] || e.s == t) continue;
            int64_t d1 = 0, d2 = 0;
            for (int a = 0; a < 3; ++a) {
                d1 += (back[a] - e.e0[a]) * (back[a] - e.e0[a]);
                d2 += (e.fwd[a] - c0[a]) * (e.fwd[a] - c0[a]);
            }
            const int64_t d = d1 < d2 ? d1 : d2;
            if ((double)d > r2) continue;
            if (best_d < 0 || d < best_d || (d == best_d && e.name < best_last)) {
                best_d = d;
                best_last = e.name;
                best_s = e.s;
            }
        }
        if (best_d >= 0) {
            used[best_s] = 1;
            cells[first].prev = best_last;
            cells[first].kind = 3;
        }
    }
    return 0;
}

}  // namespace ss4
