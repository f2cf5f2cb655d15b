// Wavelet-domain superposition (Eq.(2)), inverse Haar transform (Sec. 2, step 3) and the
// sub-hologram procedure (Sec. 2, large-scale steps 2-4) for gfx950.
//
// Tables.  A point adds the kept coefficients of one LUT table: its depth plane's, or with phase
// tables the table of its plane and of its position inside its 2^L block.  Below, "plane" means
// such a table; a point's `depth` field is its table index.
//
// Tiles.  The window is cut into 64 x 64 pixel tiles (ragged at the right and bottom edges).  With
// window origins on the 2^L grid and every table placed at the corner of its point's 2^L block,
// every coefficient a point contributes belongs to one aligned 2^L x 2^L Haar block of the window,
// so a tile's coefficients are exactly the coefficients of its own blocks.  One workgroup owns one
// tile and keeps its coefficients in LDS, block by block (each block in its own L-level Mallat
// layout, block stride BS(L)).
//
// Binning.  The points are sorted by (plane, row band) and, for every list cell (a tile or a
// square of tiles), listed when their occupied table area overlaps it.
//
// Superposition.  For a (tile, point) pair the table blocks that fall in the tile form a
// rectangle; in the sparse layout its entries are one contiguous LUT range per block row, walked
// by a wave that adds a_j * c into LDS as packed fixed-point (re, im) words with one 64-bit integer
// add; in the dense layout each wave sums whole table blocks into its own coefficients in FP32
// registers.  No global atomics touch the wavelet field.
//
// Output.  MODE_PSI writes the tile's coefficients into the Mallat layout of the window;
// MODE_FUSED inverts the tile's blocks on chip and writes pixels, so the wavelet field never
// reaches HBM.  idwt_kernel gathers a tile from a Mallat-layout field, inverts it in LDS and
// writes pixels.
#include <algorithm>
#include <cstdlib>
#include <mutex>

#include "common.hpp"

namespace cgh {
namespace {

constexpr int kT = 64;  // tile side, pixels
constexpr int kThreads = 256;       // idwt workgroup
constexpr int kTileThreads = 512;   // superposition workgroup (8 waves; four fit a CU)
constexpr int MODE_PSI = 0, MODE_FUSED = 1;

struct TileGeom {
    int64_t ox, oy;    // window origin, global pixels
    int32_t nx, ny;    // window size
    int32_t ntx, nty;  // tiles per row / column
    int32_t cell;      // point lists are kept per cell of cell x cell pixels (a square of tiles)
    int32_t nlx, nly;  // list cells per row / column
    int32_t ltx0, lty0;  // the window's first tile on the tile grid of the lists (0 unless the
                         // lists were built for a larger window holding this one)
};

// Tile handled by workgroup b: tiles go out in blocks of 32 x 32 tiles (block rows top to bottom,
// blocks left to right; edge blocks are smaller), so the tiles that are resident together cover a
// compact region and share points, depth planes and table data.  Inside a block the tiles go in
// row-major order, or with BANDS so that each XCD's tiles form a band of rows: workgroups go to the
// 8 XCDs in turn (b mod 8), each with its own L2, and XCD k takes the k-th of 8 equal runs of the
// block's row-major tiles.  Bands measured faster for the sparse superposition of grids beyond
// 4096 tiles (65536^2: 15.0 -> 14.2 ms, 16384^2: 6.32 -> 6.22 ms), slower for a single resident
// block (2048^2: 0.34 -> 0.37 ms) and for the dense superposition and the inverse; the inverse
// keeps row-major order, the dense superposition groups the tiles of a list cell (tile_of_cells).
template <bool BANDS = false>
__device__ inline void tile_of(int b, const TileGeom &g, int &ty, int &tx)
{
    constexpr int T = 32;
    const int NX = (BANDS && g.ntx * g.nty > 4096) ? 8 : 1;
    const int R = b / (T * g.ntx);                    // block row
    const int r = b - R * T * g.ntx;
    const int h = min(T, g.nty - T * R);              // its height in tiles
    const int C = r / (h * T);                        // block column
    const int i = r - C * h * T;                      // workgroup within the block
    const int w = min(T, g.ntx - T * C);              // its width in tiles
    const int run = (h * w) / NX;                     // tiles per XCD run; the rest stay in order
    const int t = i < NX * run ? (i % NX) * run + i / NX : i;
    ty = T * R + t / w;
    tx = T * C + t % w;
}

// Tile handled by workgroup b of the dense superposition when the lists are kept per cell of
// sup x sup tiles (sup >= 2) and the window is a whole number of 32 x 32-tile blocks: each group of
// 8 sup^2 consecutive workgroups takes 8 list cells, cell k of the group on XCD k (its workgroups
// are b = k, k + 8, ... of the group, as workgroups go to the XCDs in turn).  The tiles of a cell
// walk the same list in the same order at about the same time, and on one XCD they share one L2:
// a tile's table window for one point overlaps the windows its neighbours read for the points
// just before it.  Cells are taken in 32 x 32-tile blocks (as tile_of), row-major inside a block,
// so with sup = 4 XCD k works down the block's k-th column of cells.  65536^2, 40 dB selectivity:
// FP32 values 152 -> 122 ms, FP16 63 -> 49 ms (cells of 2 x 4 or 4 x 2 per XCD instead of a
// column: 132 and 125 ms FP32).  Other grids use tile_of.
__device__ inline void tile_of_cells(int b, const TileGeom &g, int &ty, int &tx)
{
    const int sup = g.cell / kT;
    if (sup < 2 || g.ntx % 32 || g.nty % 32) {
        tile_of(b, g, ty, tx);
        return;
    }
    const int per = sup * sup, cw = 32 / sup;
    const int grp = b / (8 * per), k = b % 8, j = (b % (8 * per)) / 8;
    const int cell = grp * 8 + k;
    const int blk = cell / (cw * cw), cib = cell % (cw * cw);
    const int BR = blk / (g.ntx / 32), BC = blk % (g.ntx / 32);
    ty = BR * 32 + (cib / cw) * sup + j / sup;
    tx = BC * 32 + (cib % cw) * sup + j % sup;
}

// List cells touched by the occupied part of point p's table; false if none.
__device__ inline bool footprint(const wasabi_point &p, const DepthDesc *desc, int n_tables, int L,
                                 const TileGeom &g, int &ty0, int &ty1, int &tx0, int &tx1)
{
    if (p.depth < 0 || p.depth >= n_tables) return false;
    const DepthDesc d = desc[p.depth];
    if (d.br1 <= d.br0) return false;
    const int64_t B = 1 << L;
    const int64_t xg = (int64_t)(p.x >> L) * B, yg = (int64_t)(p.y >> L) * B;  // floor to grid
    const int64_t r_org = yg - d.W / 2 - g.oy, c_org = xg - d.W / 2 - g.ox;
    const int64_t r0 = r_org + d.br0 * B, r1 = r_org + d.br1 * B;
    const int64_t c0 = c_org + d.bc0 * B, c1 = c_org + d.bc1 * B;
    if (r1 <= 0 || c1 <= 0 || r0 >= g.ny || c0 >= g.nx) return false;
    ty0 = (int)(max(r0, (int64_t)0) / g.cell);
    ty1 = (int)((min(r1, (int64_t)g.ny) - 1) / g.cell) + 1;
    tx0 = (int)(max(c0, (int64_t)0) / g.cell);
    tx1 = (int)((min(c1, (int64_t)g.nx) - 1) / g.cell) + 1;
    return true;
}

constexpr int kMaxLdsTiles = 4096;   // per-workgroup tile histograms live in LDS up to this
// ---- point sort by (plane, row band): points grouped by plane and, within a plane, by 64-row band
//      (invalid ones last).  Tile lists built from this order walk each plane's points by row, so
//      at any moment the tiles read the same horizontal band of the plane's table: the table
//      window row of a (tile, point) pair is tile_y - point_y + W/2, which then advances in step
//      across all tiles, and the band stays in L2 while they use it. ----
struct SortKey {
    int n_tables;
    int nyb;        // row bands per plane
    int64_t y0;     // row of band 0 (window origin minus the largest half table)
};

__device__ inline int sort_key(const wasabi_point &p, const SortKey &k)
{
    if (p.depth < 0 || p.depth >= k.n_tables) return k.n_tables * k.nyb;
    int64_t b = ((int64_t)p.y - k.y0) >> 6;
    b = b < 0 ? 0 : (b >= k.nyb ? k.nyb - 1 : b);
    return p.depth * k.nyb + (int)b;
}

// Zeroes n 32-bit words.  The counters of the binning and of plane pacing are cleared with this
// kernel rather than a memset, so that the path can be captured into a HIP graph and replayed.
__global__ __launch_bounds__(256) void zero_words_kernel(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0u;
}

int zero_words(void *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return CGH_OK;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_words_kernel, dim3(grid), dim3(256), 0, s, (uint32_t *)p, n);
    CGH_CHECK_LAUNCH("zero_words_kernel");
    return CGH_OK;
}

// ---- stable radix sort (least significant digit first) -----------------------------------------
// Each pass is a stable counting sort on `bits` bits of an integer key.  Block b takes `per`
// consecutive items: it counts their digits into column b of a digit-major matrix, whose
// exclusive scan gives every (digit, block) its output range; the block then writes its items in
// input order, a round of 256 at a time: a lane's rank among the lanes of its wave with the same
// digit comes from one ballot per key bit, the waves before it add their counts (kept in LDS per
// wave and digit), and a running offset per digit carries the rounds.  Equal keys keep their input
// order, so the sorted order -- and every sum taken in it later -- does not depend on timing.
constexpr int kSortThreads = 256;   // 4 waves
constexpr int kSortMaxBits = 12;    // digits per pass: at most 4096 (48 KiB of LDS in the scatter)
constexpr int kSortPrefetch = 8;    // rounds whose items a scatter thread loads at once

struct PointKey {                   // points by (plane, row band) bin
    using T = wasabi_point;
    static constexpr bool kPair = false;
    SortKey k;
    __device__ int operator()(const wasabi_point &p) const { return sort_key(p, k); }
};

struct PairKey {                    // (list cell << 32 | point) pairs by list cell
    using T = unsigned long long;
    static constexpr bool kPair = true;
    __device__ int operator()(unsigned long long v) const { return (int)(v >> 32); }
};

template <class K>
__global__ __launch_bounds__(kSortThreads) void radix_count_kernel(const typename K::T *in, int64_t n,
                                                                   const int64_t *n_dev, K key, int shift,
                                                                   int bits, int64_t per, int nblk,
                                                                   int32_t *mat)
{
    extern __shared__ int hist[];
    const int D = 1 << bits;
    for (int i = threadIdx.x; i < D; i += kSortThreads) hist[i] = 0;
    __syncthreads();
    if (n_dev) n = min(n, *n_dev);
    const int64_t j0 = (int64_t)blockIdx.x * per, j1 = min(n, j0 + per);
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kSortThreads) atomicAdd(&hist[(key(in[j]) >> shift) & (D - 1)], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < D; i += kSortThreads) mat[(int64_t)i * nblk + blockIdx.x] = hist[i];
}

// out_low: when not NULL the items' low 32 bits go there instead of the items to `out` (the last
// pass of the pair sort writes the point indices of the lists directly).
template <class K>
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(const typename K::T *in, int64_t n,
                                                                     const int64_t *n_dev, K key, int shift,
                                                                     int bits, int64_t per, int nblk,
                                                                     const int64_t *moff, typename K::T *out,
                                                                     int32_t *out_low)
{
    extern __shared__ int sh[];
    const int D = 1 << bits;
    int *run = sh;                                        // next output position of each digit
    unsigned short *wcnt = (unsigned short *)(sh + D);    // [4][D]: items per wave and digit this round
    for (int i = threadIdx.x; i < D; i += kSortThreads) {
        run[i] = (int)moff[(int64_t)i * nblk + blockIdx.x];
#pragma unroll
        for (int w = 0; w < 4; ++w) wcnt[w * D + i] = 0;
    }
    __syncthreads();
    if (n_dev) n = min(n, *n_dev);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t j0 = (int64_t)blockIdx.x * per, j1 = min(n, j0 + per);
    // the items of kSortPrefetch rounds are loaded at once, so the rounds wait on memory once
    typename K::T pre[kSortPrefetch];
    for (int64_t base = j0; base < j1; base += kSortThreads) {
        const int r = (int)(((base - j0) / kSortThreads) % kSortPrefetch);
        if (r == 0) {
#pragma unroll
            for (int q = 0; q < kSortPrefetch; ++q) {
                const int64_t jq = base + (int64_t)q * kSortThreads + threadIdx.x;
                if (jq < j1) pre[q] = in[jq];
            }
        }
        const int64_t j = base + threadIdx.x;
        const bool act = j < j1;
        typename K::T v{};
        int dg = 0;
        if (act) {
            // the round's item, picked from the prefetched ones with indices fixed at compile time
#pragma unroll
            for (int q = 0; q < kSortPrefetch; ++q)
                if (q == r) v = pre[q];
            dg = (key(v) >> shift) & (D - 1);
        }
        // lanes of this wave with the same digit
        unsigned long long peers = __ballot(act);
        for (int b = 0; b < bits; ++b) {
            const bool bit = (dg >> b) & 1;
            const unsigned long long bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const bool leader = act && (peers & below) == 0;
        const int cnt = __popcll(peers);
        if (leader) wcnt[wave * D + dg] = (unsigned short)cnt;
        __syncthreads();
        if (act) {
            int pos = run[dg] + __popcll(peers & below);
            for (int w = 0; w < wave; ++w) pos += wcnt[w * D + dg];
            if constexpr (K::kPair) {
                if (out_low) out_low[pos] = (int32_t)(uint32_t)v;
                else out[pos] = v;
            } else {
                out[pos] = v;
            }
        }
        __syncthreads();
        if (leader) {
            atomicAdd(&run[dg], cnt);
            wcnt[wave * D + dg] = 0;
        }
        __syncthreads();
    }
}

// ---- per-cell point lists (counting sort by list cell; a cell is a square of tiles) -------------------------------------------
template <bool LDS>
__global__ __launch_bounds__(256) void bin_count_kernel(const wasabi_point *pts, int64_t n,
                                                        const DepthDesc *desc, int n_tables, int L,
                                                        TileGeom g, int32_t *counts)
{
    __shared__ int hist[LDS ? kMaxLdsTiles : 1];
    const int ntiles = g.nlx * g.nly;
    if (LDS) {
        for (int i = threadIdx.x; i < ntiles; i += 256) hist[i] = 0;
        __syncthreads();
    }
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int ty0, ty1, tx0, tx1;
    if (j < n && footprint(pts[j], desc, n_tables, L, g, ty0, ty1, tx0, tx1)) {
        for (int ty = ty0; ty < ty1; ++ty)
            for (int tx = tx0; tx < tx1; ++tx) {
                if (LDS) atomicAdd(&hist[ty * g.nlx + tx], 1);
                else atomicAdd(&counts[(int64_t)ty * g.nlx + tx], 1);
            }
    }
    if (LDS) {
        __syncthreads();
        for (int i = threadIdx.x; i < ntiles; i += 256)
            if (hist[i]) atomicAdd(&counts[i], hist[i]);
    }
}

template <bool LDS>
__global__ __launch_bounds__(256) void bin_fill_kernel(const wasabi_point *pts, int64_t n,
                                                       const DepthDesc *desc, int n_tables, int L,
                                                       TileGeom g, unsigned long long *cursor,
                                                       int32_t *list)
{
    __shared__ int cnt[LDS ? kMaxLdsTiles : 1];
    __shared__ unsigned long long base[LDS ? kMaxLdsTiles : 1];
    const int ntiles = g.nlx * g.nly;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int ty0 = 0, ty1 = 0, tx0 = 0, tx1 = 0;
    const bool has = j < n && footprint(pts[j], desc, n_tables, L, g, ty0, ty1, tx0, tx1);
    if (LDS) {
        for (int i = threadIdx.x; i < ntiles; i += 256) cnt[i] = 0;
        __syncthreads();
        if (has)
            for (int ty = ty0; ty < ty1; ++ty)
                for (int tx = tx0; tx < tx1; ++tx) atomicAdd(&cnt[ty * g.nlx + tx], 1);
        __syncthreads();
        for (int i = threadIdx.x; i < ntiles; i += 256) {
            if (cnt[i]) base[i] = atomicAdd(&cursor[i], (unsigned long long)cnt[i]);
            cnt[i] = 0;
        }
        __syncthreads();
    }
    if (has)
        for (int ty = ty0; ty < ty1; ++ty)
            for (int tx = tx0; tx < tx1; ++tx) {
                const int t = ty * g.nlx + tx;
                unsigned long long slot;
                if (LDS) slot = base[t] + (unsigned long long)atomicAdd(&cnt[t], 1);
                else slot = atomicAdd(&cursor[(int64_t)ty * g.nlx + tx], 1ull);
                list[slot] = (int32_t)j;
            }
}

// Deterministic lists beyond kMaxLdsTiles cells: every sorted point writes its (cell, point) pairs
// in cell order at its own offset (an exclusive scan of its cell count), and a stable sort of the
// pairs by cell then leaves each cell's list in sorted-point order.
__global__ __launch_bounds__(256) void point_cells_kernel(const wasabi_point *pts, int64_t n,
                                                          const DepthDesc *desc, int n_tables, int L,
                                                          TileGeom g, int32_t *cells)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int ty0, ty1, tx0, tx1;
    cells[j] = footprint(pts[j], desc, n_tables, L, g, ty0, ty1, tx0, tx1) ? (ty1 - ty0) * (tx1 - tx0) : 0;
}

__global__ __launch_bounds__(256) void pair_fill_kernel(const wasabi_point *pts, int64_t n,
                                                        const DepthDesc *desc, int n_tables, int L,
                                                        TileGeom g, const int64_t *poff,
                                                        unsigned long long *pairs)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int ty0, ty1, tx0, tx1;
    if (j >= n || !footprint(pts[j], desc, n_tables, L, g, ty0, ty1, tx0, tx1)) return;
    int64_t at = poff[j];
    for (int ty = ty0; ty < ty1; ++ty)
        for (int tx = tx0; tx < tx1; ++tx)
            pairs[at++] = ((unsigned long long)(ty * g.nlx + tx) << 32) | (unsigned long long)(uint32_t)j;
}

// Ordered lists: chunk w (`cpts` consecutive sorted points) writes its per-tile counts to column w of a
// tile-major matrix; the exclusive scan of that matrix gives each chunk its slice of every tile's
// list, in chunk order.  Inside a chunk one wave takes the points one after another (lanes spread
// over the point's tiles), so every tile's list keeps the sorted point order exactly.
constexpr int kChunk = 64;      // threads per workgroup, and the most points per chunk

// Points per chunk: 32 for small point sets (twice the workgroups, half the points each walks in
// turn), else 64 (half the matrix).
inline int chunk_pts(int64_t n) { return n <= 65536 ? 32 : kChunk; }

__global__ __launch_bounds__(kChunk) void bin_count_matrix_kernel(const wasabi_point *pts, int64_t n,
                                                                  const DepthDesc *desc, int n_tables,
                                                                  int L, TileGeom g, int nwg, int cpts,
                                                                  int32_t *mat)
{
    __shared__ int hist[kMaxLdsTiles];
    const int ntiles = g.nlx * g.nly;
    for (int i = threadIdx.x; i < ntiles; i += kChunk) hist[i] = 0;
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * cpts + threadIdx.x;
    int ty0, ty1, tx0, tx1;
    if (threadIdx.x < cpts && j < n && footprint(pts[j], desc, n_tables, L, g, ty0, ty1, tx0, tx1))
        for (int ty = ty0; ty < ty1; ++ty)
            for (int tx = tx0; tx < tx1; ++tx) atomicAdd(&hist[ty * g.nlx + tx], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < ntiles; i += kChunk) mat[(int64_t)i * nwg + blockIdx.x] = hist[i];
}

__global__ __launch_bounds__(kChunk) void bin_fill_matrix_kernel(const wasabi_point *pts, int64_t n,
                                                                 const DepthDesc *desc, int n_tables,
                                                                 int L, TileGeom g, int nwg, int cpts,
                                                                 const int64_t *moff, int32_t *list)
{
    // next free list position of this workgroup's segment in every tile's list (all loads in
    // flight at once, so the point loop below only reads on-chip memory)
    __shared__ int64_t pos[kMaxLdsTiles];
    __shared__ int fp[kChunk][4];
    const int ntiles = g.nlx * g.nly;
    for (int i = threadIdx.x; i < ntiles; i += kChunk) pos[i] = moff[(int64_t)i * nwg + blockIdx.x];
    const int64_t j0 = (int64_t)blockIdx.x * cpts;
    const int np = (int)min((int64_t)cpts, n - j0);
    {
        int ty0 = 0, ty1 = 0, tx0 = 0, tx1 = 0;
        if (threadIdx.x < np && !footprint(pts[j0 + threadIdx.x], desc, n_tables, L, g, ty0, ty1, tx0, tx1))
            ty0 = ty1 = tx0 = tx1 = 0;
        fp[threadIdx.x][0] = ty0;
        fp[threadIdx.x][1] = ty1;
        fp[threadIdx.x][2] = tx0;
        fp[threadIdx.x][3] = tx1;
    }
    __syncthreads();
    // points in order (the lists stay in sorted-point order); the threads share a point's tiles
    for (int q = 0; q < np; ++q) {
        const int ty0 = fp[q][0], ty1 = fp[q][1], tx0 = fp[q][2], tx1 = fp[q][3];
        const int w = tx1 - tx0, cells = (ty1 - ty0) * w;
        for (int c = threadIdx.x; c < cells; c += kChunk) {
            const int t = (ty0 + c / w) * g.nlx + tx0 + c % w;
            list[pos[t]++] = (int32_t)(j0 + q);
        }
        __syncthreads();
    }
}

// Per list cell: B = sum over its points of |a_j| max|c|_plane(j), the bound from which the sparse
// kernel sets its fixed-point scale (every tile of the cell sees a subset of these points).
__global__ __launch_bounds__(256) void cell_bound_kernel(const wasabi_point *pts, const int32_t *list,
                                                         const int64_t *off, const DepthDesc *desc,
                                                         double *bound)
{
    __shared__ double red[4];
    const int64_t p0 = off[blockIdx.x], p1 = off[blockIdx.x + 1];
    double b = 0.0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) {
        const wasabi_point pt = pts[list[p]];
        b += (double)fabsf(pt.a) * (double)desc[pt.depth].cmax;
    }
    for (int o = 32; o > 0; o >>= 1) b += __shfl_down(b, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) bound[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void gather_tile_off_kernel(const int64_t *moff, int64_t ntiles, int nwg, int64_t *off)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= ntiles) off[t] = moff[t * nwg];
}

// ---- exclusive scan of int32 counts into int64 offsets (n + 1 values) ----------------------
__device__ inline int64_t block_incl_scan(int64_t v, int64_t *wave_sums, int64_t &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    if (lane == 63) wave_sums[wave] = v;
    __syncthreads();
    int64_t off = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        const int64_t s = wave_sums[w];
        off += (w < wave) ? s : 0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return v + off;
}

__global__ __launch_bounds__(1024) void scan_local_kernel(const int32_t *counts, int64_t n,
                                                          int64_t *off, int64_t *bsum)
{
    __shared__ int64_t ws[16];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const int64_t v = i < n ? counts[i] : 0;
    int64_t tot;
    const int64_t incl = block_incl_scan(v, ws, tot);
    if (i < n) off[i] = incl - v;
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of a short count array by one workgroup: off[i] for i < n, off[n] = the total,
// and the same offsets into `copy` unless it is NULL.
__global__ __launch_bounds__(1024) void scan_small_kernel(const int32_t *counts, int64_t n, int64_t *off,
                                                          unsigned long long *copy)
{
    __shared__ int64_t ws[16];
    int64_t carry = 0;
    for (int64_t base = 0; base < n; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < n ? counts[i] : 0;
        int64_t tot;
        const int64_t excl = carry + block_incl_scan(v, ws, tot) - v;
        if (i < n) {
            off[i] = excl;
            if (copy) copy[i] = (unsigned long long)excl;
        }
        carry += tot;
    }
    if (threadIdx.x == 0) off[n] = carry;
}

__global__ __launch_bounds__(1024) void scan_sums_kernel(int64_t *bsum, int64_t nb, int64_t *total_out)
{
    __shared__ int64_t ws[16];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < nb ? bsum[i] : 0;
        int64_t tot;
        const int64_t incl = block_incl_scan(v, ws, tot);
        if (i < nb) bsum[i] = carry + incl - v;
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ void scan_add_kernel(int64_t *off, int64_t n, const int64_t *bsum)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) off[i] += bsum[i / 1024];
}

// ---- tile kernels ---------------------------------------------------------------------------
struct TileArgs {
    const DepthDesc *desc;
    const int32_t *blk_off;
    const void *values;
    const uint16_t *keys;
    const int32_t *wkeys;      // sparse layout: each entry's byte offset in the tile buffer (L >= 3)
    const wasabi_point *pts;
    const int64_t *tile_off;
    const int32_t *tile_pts;
    const double *cell_bound;  // per list cell: sum of |a| max|c| over its points
    TileGeom g;
    const float2 *in;  // idwt: Mallat-layout field of the window (contiguous, row stride nx)
    float2 *out;       // MODE_PSI: Mallat field (row stride nx); otherwise pixels (row stride ld)
    int64_t ld;
    const void *dense;          // dense layout values (or NULL)
    int64_t dense_zero;         // first of kDenseZero zero values in `dense`
    const DenseRow *dense_rows; // dense layout block-row spans
    int n_tables;
    int *plane_done;            // plane pacing: tiles that finished plane d (NULL = off)
    int pace_slack;             // a tile starts plane d once all tiles finished plane d - slack
    int stream_psi;             // MODE_PSI: the Mallat field is written past the caches
    int accumulate;             // MODE_PSI: add to the field's values instead of overwriting them
};

template <int L>
struct TileShape {
    static constexpr int B = 1 << L;
    static constexpr int TB = kT / B;             // blocks per tile side
    static constexpr int BS = block_stride(L);    // LDS floats per block
    static constexpr int ROW = TB * BS + row_pad(L);  // LDS floats per block row
    static constexpr int N = TB * ROW;            // LDS floats per plane (re or im)
};

template <int VT>
__device__ inline float2 load_value(const void *values, int64_t i)
{
    if (VT == CGH_F32) return ((const float2 *)values)[i];
    const uint32_t w = ((const uint32_t *)values)[i];
    if (VT == CGH_F16) {
        _Float16 lo, hi;
        const uint16_t l16 = (uint16_t)(w & 0xffff), h16 = (uint16_t)(w >> 16);
        __builtin_memcpy(&lo, &l16, 2);
        __builtin_memcpy(&hi, &h16, 2);
        return make_float2((float)lo, (float)hi);
    }
    return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
}

// 16-byte loads of stored values: E consecutive complex values (E = 2 for FP32, 4 for FP16/BF16).
template <int VT>
struct Wide {
    static constexpr int E = VT == CGH_F32 ? 2 : 4;
};

template <int VT>
__device__ inline float2 unpack_value(uint32_t w)
{
    if (VT == CGH_F16) {
        _Float16 lo, hi;
        const uint16_t l16 = (uint16_t)(w & 0xffff), h16 = (uint16_t)(w >> 16);
        __builtin_memcpy(&lo, &l16, 2);
        __builtin_memcpy(&hi, &h16, 2);
        return make_float2((float)lo, (float)hi);
    }
    return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
}

// values[i .. i + E) (i a multiple of E) into out[0 .. E)
template <int VT>
__device__ inline void load_wide(const void *values, int64_t i, float2 *out)
{
    if constexpr (VT == CGH_F32) {
        const float4 q = *(const float4 *)((const float2 *)values + i);
        out[0] = make_float2(q.x, q.y);
        out[1] = make_float2(q.z, q.w);
    } else {
        const uint4 q = *(const uint4 *)((const uint32_t *)values + i);
        out[0] = unpack_value<VT>(q.x);
        out[1] = unpack_value<VT>(q.y);
        out[2] = unpack_value<VT>(q.z);
        out[3] = unpack_value<VT>(q.w);
    }
}

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

// Stores one complex value of a Mallat field through the caches or (nt) past them; with `acc` the
// value is added to the one already there.
__device__ inline void put2(float2 *p, float2 v, bool nt, bool acc)
{
    if (acc) {
        const float2 o = *p;
        v = make_float2(o.x + v.x, o.y + v.y);
    }
    if (nt)
        __builtin_nontemporal_store((v2f){v.x, v.y}, reinterpret_cast<v2f *>(p));
    else
        *p = v;
}

// Loads the tile's coefficients from the window's Mallat field (rows of nx) into the tile buffer.
// The level / band loops are unrolled, so every slot of the register staging arrays is known at
// compile time, and every load of a thread is issued before any of its stores to LDS.
template <int L, int NT>
__device__ inline void tile_mallat_load(float *sre, float *sim, const float2 *field, const TileGeom &g,
                                        int ty, int tx, int th, int tw)
{
    using S = TileShape<L>;
    constexpr int K = 3 * ((kT * kT / 4 + NT - 1) / NT) * L + (kT * kT / (1 << (2 * L)) + NT - 1) / NT;
    float2 v[K];
    int at[K];
    int slot = 0;
#pragma unroll
    for (int l = 1; l <= L; ++l) {
        const int wf = kT >> l, h = S::B >> l;
#pragma unroll
        for (int band = 1; band <= 3; ++band) {
            const int64_t row0 = (band & 2) ? (g.ny >> l) : 0, col0 = (band & 1) ? (g.nx >> l) : 0;
#pragma unroll
            for (int i0 = 0; i0 < wf * wf; i0 += NT, ++slot) {
                const int i = i0 + threadIdx.x, m = i / wf, n = i % wf;
                at[slot] = -1;
                if (i < wf * wf && m < (th >> l) && n < (tw >> l)) {
                    const int code = (((band & 2) ? h : 0) + (m & (h - 1))) * S::B + ((band & 1) ? h : 0) + (n & (h - 1));
                    at[slot] = (m / h) * S::ROW + (n / h) * S::BS + code;
                    v[slot] = field[(row0 + (int64_t)ty * wf + m) * g.nx + col0 + (int64_t)tx * wf + n];
                }
            }
        }
    }
    {
        constexpr int wf = kT >> L;
#pragma unroll
        for (int i0 = 0; i0 < wf * wf; i0 += NT, ++slot) {
            const int i = i0 + threadIdx.x, m = i / wf, n = i % wf;
            at[slot] = -1;
            if (i < wf * wf && m < (th >> L) && n < (tw >> L)) {
                at[slot] = m * S::ROW + n * S::BS;
                v[slot] = field[((int64_t)ty * wf + m) * g.nx + (int64_t)tx * wf + n];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (k < slot && at[k] >= 0) {
            sre[at[k]] = v[k].x;
            sim[at[k]] = v[k].y;
        }
}

// Moves the tile's coefficients between LDS and the window's Mallat layout (rows of nx).
template <int L, bool TO_LDS, int NT>
__device__ inline void tile_mallat_io(float *sre, float *sim, float2 *field, const TileGeom &g,
                                      int ty, int tx, int th, int tw, bool add = false)
{
    using S = TileShape<L>;
    const int64_t nx = g.nx;
#pragma unroll
    for (int l = 1; l <= L; ++l) {
        const int wf = kT >> l;          // band extent of a full tile at level l
        const int h = S::B >> l;         // band extent inside one block
        const int hb = th >> l, wb = tw >> l;
        for (int band = 1; band <= 3; ++band) {
            const int64_t row0 = (band & 2) ? (g.ny >> l) : 0, col0 = (band & 1) ? (g.nx >> l) : 0;
            for (int i = threadIdx.x; i < wf * wf; i += NT) {
                const int m = i / wf, n = i % wf;
                if (m >= hb || n >= wb) continue;
                const int code = (((band & 2) ? h : 0) + (m & (h - 1))) * S::B + ((band & 1) ? h : 0) + (n & (h - 1));
                const int at = (m / h) * S::ROW + (n / h) * S::BS + code;
                float2 *f = field + (row0 + (int64_t)ty * wf + m) * nx + col0 + (int64_t)tx * wf + n;
                if (TO_LDS) {
                    const float2 v = *f;
                    sre[at] = v.x;
                    sim[at] = v.y;
                } else {
                    put2(f, make_float2(sre[at], sim[at]), false, add);
                }
            }
        }
    }
    {
        const int wf = kT >> L;
        const int hb = th >> L, wb = tw >> L;
        for (int i = threadIdx.x; i < wf * wf; i += NT) {
            const int m = i / wf, n = i % wf;
            if (m >= hb || n >= wb) continue;
            const int at = m * S::ROW + n * S::BS;
            float2 *f = field + ((int64_t)ty * wf + m) * nx + (int64_t)tx * wf + n;
            if (TO_LDS) {
                const float2 v = *f;
                sre[at] = v.x;
                sim[at] = v.y;
            } else {
                put2(f, make_float2(sre[at], sim[at]), false, add);
            }
        }
    }
}

// In-LDS inverse Haar of every block of the tile, then the pixels go to out (row stride ld).  With
// STREAM the pixels are written two to a 16-byte non-temporal store: the fused superposition's
// hologram is not read again here, and streaming it past the caches leaves the L2 to the table
// data (65536^2, 40 dB selectivity: FP32 values 95.0 -> 92.6 ms, FP16 49.7 -> 47.8 ms; 2048^2
// 1.29 -> 1.26 ms).
template <int L, int NT, bool STREAM = false>
__device__ inline void tile_inverse_and_store(float *sre, float *sim, float2 *out, int64_t ld,
                                              int ty, int tx, int th, int tw)
{
    using S = TileShape<L>;
    constexpr int MAXQ = (kT * kT / 4 + NT - 1) / NT;
#pragma unroll
    for (int l = L; l >= 1; --l) {
        const int h = S::B >> l;           // S^(l) extent inside a block
        const int per = h * h;
        const int nq = (kT >> l) * (kT >> l);
        float r[MAXQ][4], im[MAXQ][4];
        int base[MAXQ], mm[MAXQ], nn[MAXQ];
#pragma unroll
        for (int k = 0; k < MAXQ; ++k) {
            const int qi = threadIdx.x + NT * k;
            if (qi < nq) {
                const int blk = qi / per, w = qi % per;
                const int m = w / h, n = w % h;
                const int b = (blk / S::TB) * S::ROW + (blk % S::TB) * S::BS;
                base[k] = b;
                mm[k] = m;
                nn[k] = n;
                const int s0 = b + m * S::B + n, s1 = s0 + h, s2 = s0 + h * S::B, s3 = s2 + h;
                r[k][0] = sre[s0]; r[k][1] = sre[s1]; r[k][2] = sre[s2]; r[k][3] = sre[s3];
                im[k][0] = sim[s0]; im[k][1] = sim[s1]; im[k][2] = sim[s2]; im[k][3] = sim[s3];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < MAXQ; ++k) {
            const int qi = threadIdx.x + NT * k;
            if (qi < nq) {
                const int a00 = base[k] + (2 * mm[k]) * S::B + 2 * nn[k];
                const int a10 = a00 + S::B;
                const float Sr = r[k][0], Hr = r[k][1], Vr = r[k][2], Dr = r[k][3];
                const float Si = im[k][0], Hi = im[k][1], Vi = im[k][2], Di = im[k][3];
                sre[a00] = (Sr + Hr + Vr + Dr) * 0.5f;
                sre[a00 + 1] = (Sr - Hr + Vr - Dr) * 0.5f;
                sre[a10] = (Sr + Hr - Vr - Dr) * 0.5f;
                sre[a10 + 1] = (Sr - Hr - Vr + Dr) * 0.5f;
                sim[a00] = (Si + Hi + Vi + Di) * 0.5f;
                sim[a00 + 1] = (Si - Hi + Vi - Di) * 0.5f;
                sim[a10] = (Si + Hi - Vi - Di) * 0.5f;
                sim[a10 + 1] = (Si - Hi - Vi + Di) * 0.5f;
            }
        }
        __syncthreads();
    }
    if constexpr (STREAM) {
        const bool wide = ((reinterpret_cast<uintptr_t>(out) | (uintptr_t)ld * sizeof(float2)) & 15) == 0;
        for (int i = threadIdx.x; i < kT * kT / 2; i += NT) {
            const int rr = i / (kT / 2), cc = 2 * (i % (kT / 2));
            if (rr >= th || cc >= tw) continue;
            const int at = (rr >> L) * S::ROW + (cc >> L) * S::BS + (rr & (S::B - 1)) * S::B + (cc & (S::B - 1));
            float2 *o = out + ((int64_t)ty * kT + rr) * ld + (int64_t)tx * kT + cc;
            if (wide) {
                __builtin_nontemporal_store((v4f){sre[at], sim[at], sre[at + 1], sim[at + 1]}, reinterpret_cast<v4f *>(o));
            } else {
                __builtin_nontemporal_store((v2f){sre[at], sim[at]}, reinterpret_cast<v2f *>(o));
                __builtin_nontemporal_store((v2f){sre[at + 1], sim[at + 1]}, reinterpret_cast<v2f *>(o + 1));
            }
        }
        return;
    }
    for (int i = threadIdx.x; i < kT * kT; i += NT) {
        const int rr = i / kT, cc = i % kT;
        if (rr >= th || cc >= tw) continue;
        const int at = (rr >> L) * S::ROW + (cc >> L) * S::BS + (rr & (S::B - 1)) * S::B + (cc & (S::B - 1));
        out[((int64_t)ty * kT + rr) * ld + (int64_t)tx * kT + cc] = make_float2(sre[at], sim[at]);
    }
}

// Fixed-point accumulation.  LDS float atomics are slow on this GPU, integer ones are not, so each
// term a_j * c is formed exactly in FP64 (a product of two FP32 values), rounded once to the grid
// 2^-s, and added as an integer.  Integer sums are exact and independent of the order of the adds.
// s is chosen per tile from the bound B_t = sum_j |a_j| max|c|_plane(j) over the tile's points
// (each point adds at most one term to any coefficient): with B_t < 2^e and s = 30 - e, every
// scaled partial and final sum stays below 2^31 in magnitude.  Rounding uses the FP64 "magic
// number" 1.5 * 2^52: for |y| < 2^31 the low 32 bits of y + 1.5 * 2^52 are round-to-nearest-even(y)
// in two's complement.
// A coefficient's 8-byte LDS slot holds its real sum in the low 32 bits and its imaginary sum in
// the high 32 bits, each added with its own 32-bit atomic (measured as fast as packing both parts
// into one 64-bit add, and it needs no unpacking of the sums).
constexpr double kMagic = 6755399441055744.0;  // 1.5 * 2^52

__device__ inline int to_fixed(float v, double scaled_amp)
{
    return __double2loint(fma((double)v, scaled_amp, kMagic));
}

// Adds a_j * v (scaled_amp = a_j 2^s) to the slot at byte address wbyte of the tile buffer.
__device__ inline void lds_add(unsigned long long *acc, int wbyte, float2 v, double scaled_amp)
{
    unsigned *w = reinterpret_cast<unsigned *>(reinterpret_cast<char *>(acc) + wbyte);
    atomicAdd(w, (unsigned)to_fixed(v.x, scaled_amp));
    atomicAdd(w + 1, (unsigned)to_fixed(v.y, scaled_amp));
}

// Adds the kept coefficients of one (tile, point) pair into the tile's LDS accumulators, for L <= 2
// (more than 8 block rows per pair; walk_pairs takes L >= 3).  Called by a whole wave with uniform
// arguments: the pair's table blocks inside the tile are `nrows` block rows; row r's entries are
// the contiguous LUT range [rstart_r, rstart_r + rcount_r) (held by lane r) and land at LDS
// element dst0 + r * ROW + key.  Each row is walked U x 64 entries at a time with all loads issued
// before the LDS adds; lanes past the end of a row are masked off.
template <int L, int VT>
__device__ inline void add_pair(unsigned long long *acc, const void *values, const uint16_t *keys,
                                int eb, int dst0, int nrows, double scaled_amp, int rstart,
                                int rcount)
{
    using S = TileShape<L>;
    const int lane = threadIdx.x & 63;
    constexpr int U = 4;
    for (int r = 0; r < nrows; ++r) {
        const int rs = __builtin_amdgcn_readlane(rstart, r);
        const int rc = __builtin_amdgcn_readlane(rcount, r);
        const int d = dst0 + r * S::ROW;
        const int64_t first = (int64_t)eb + rs;
        const uint16_t *kp = keys + first;
        for (int c = 0; c < rc; c += 64 * U) {
            float2 v[U];
            int k[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = c + 64 * u + lane;
                if (e < rc) {
                    v[u] = load_value<VT>(values, first + e);
                    k[u] = kp[e];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = c + 64 * u + lane;
                if (e < rc) lds_add(acc, (d + k[u]) * (int)sizeof(unsigned long long), v[u], scaled_amp);
            }
        }
    }
}

// Walks a batch of (tile, point) pairs (lane k holds pair k's metadata) for L >= 3 (at most 8
// block rows per pair).  The row ranges of all pairs of the batch are loaded at once, so a pair
// waits only for its own entries; a pair's rows are walked as one flat range of entries (row r
// owns [ex_r, ex_r + count_r)), 64 lanes x 2 entries per step with all loads of a step issued
// before its adds, and a last step of one entry per lane when at most 64 entries are left.
// The kernel is bound by VALU issue here, so the per-entry work is kept small: entries are
// addressed by 32-bit offsets from the pair's plane (the 16-bit keys keep a table side below
// 8192 pixels, so a table holds fewer than 2^26 entries), and
// lanes past the end are masked off rather than given neutral values.
template <int L>
struct PairStep {
    using S = TileShape<L>;
    int ex[S::TB], off[S::TB];
    int total, baseb;       // baseb: LDS byte address of the table's block (0, 0) in this tile
    const char *vals;       // the plane's first stored value
    const int32_t *wkeys;   // and the byte offset of its first entry
    double sa;
};

template <int L, int VT>
__device__ inline void pair_setup(PairStep<L> &P, int k, const int *m_rs, const int *m_rcp, int m_eb,
                                  int m_base, float m_amp, int shift, const TileArgs &a)
{
    using S = TileShape<L>;
    constexpr int vbytes = VT == CGH_F32 ? 8 : 4;
    P.total = 0;
#pragma unroll
    for (int r = 0; r < S::TB; ++r) {
        const unsigned rcp = (unsigned)__builtin_amdgcn_readlane(m_rcp[r / 2], k);
        P.ex[r] = P.total;
        P.off[r] = __builtin_amdgcn_readlane(m_rs[r], k) - P.total;
        P.total += (int)((r & 1) ? rcp >> 16 : rcp & 0xffff);
    }
    const int eb = __builtin_amdgcn_readlane(m_eb, k);
    P.vals = (const char *)a.values + (int64_t)eb * vbytes;
    P.wkeys = a.wkeys + eb;
    P.baseb = __builtin_amdgcn_readlane(m_base, k) * (int)sizeof(unsigned long long);
    P.sa = ldexp((double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(m_amp), k)), shift);
}

// The entry offset of the row holding entry e: a select chain over rows R, R + 1, ... (indices
// fixed at compile time, so that the rows' values stay in registers rather than in an indexed
// private array).
template <int L, int R>
__device__ inline void row_select(const PairStep<L> &P, int e, int &o)
{
    if constexpr (R < TileShape<L>::TB) {
        if (e >= P.ex[R]) o = P.off[R];
        row_select<L, R + 1>(P, e, o);
    }
}

// Entry e of the pair (0 <= e < total): its stored value, and the byte address of its LDS word
// (the entry's own offset from the table's block (0, 0), which carries its block row, plus where
// that block sits in the tile).
template <int L, int VT>
__device__ inline void pair_entry(const PairStep<L> &P, int e, float2 &v, int &wbyte)
{
    int o = P.off[0];
    row_select<L, 1>(P, e, o);
    const uint32_t rel = (uint32_t)(e + o);  // entry index within the plane's table
    if constexpr (VT == CGH_F32) {
        v = *reinterpret_cast<const float2 *>(P.vals + (rel << 3));
    } else {
        const uint32_t w = *reinterpret_cast<const uint32_t *>(P.vals + (rel << 2));
        if constexpr (VT == CGH_F16) {
            _Float16 lo, hi;
            const uint16_t l16 = (uint16_t)(w & 0xffff), h16 = (uint16_t)(w >> 16);
            __builtin_memcpy(&lo, &l16, 2);
            __builtin_memcpy(&hi, &h16, 2);
            v = make_float2((float)lo, (float)hi);
        } else {
            v = make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
        }
    }
    wbyte = P.baseb + *reinterpret_cast<const int32_t *>(reinterpret_cast<const char *>(P.wkeys) + (rel << 2));
}

template <int L, int VT>
__device__ inline void walk_pairs(unsigned long long *acc, const TileArgs &a, int cnt, int m_nrows,
                                  int m_bo, int m_nb, int m_bc0, int m_bc1, int m_eb, int m_base,
                                  float m_amp, int shift)
{
    using S = TileShape<L>;
    const int lane = threadIdx.x & 63;
    // all loads issued together: rows past the pair's last re-read its first row, counted as empty
    // (32-bit byte offsets from the array's base: the library keeps blk_off below 2^30 entries)
    int m_rs[S::TB], m_rc[S::TB];
    const char *bo = reinterpret_cast<const char *>(a.blk_off);
#pragma unroll
    for (int r = 0; r < S::TB; ++r) {
        const uint32_t row = (uint32_t)(m_bo + (r < m_nrows ? r : 0) * m_nb);
        m_rs[r] = *reinterpret_cast<const int32_t *>(bo + ((row + (uint32_t)m_bc0) << 2));
        m_rc[r] = *reinterpret_cast<const int32_t *>(bo + ((row + (uint32_t)m_bc1) << 2));
    }
    int m_tot = 0;
#pragma unroll
    for (int r = 0; r < S::TB; ++r) {
        m_rc[r] = r < m_nrows ? m_rc[r] - m_rs[r] : 0;
        m_tot += m_rc[r];
    }
    // row counts two to a register (a row of a pair holds at most 64 2^L <= 4096 entries)
    int m_rcp[(S::TB + 1) / 2];
#pragma unroll
    for (int r = 0; r < S::TB; r += 2) m_rcp[r / 2] = m_rc[r] | (r + 1 < S::TB ? m_rc[r + 1] << 16 : 0);
    // the pairs with at least one entry, in order
    auto next_pair = [&](int k) {
        while (k < cnt && __builtin_amdgcn_readlane(m_tot, k) == 0) ++k;
        return k;
    };
    for (int k = next_pair(0); k < cnt; k = next_pair(k + 1)) {
        PairStep<L> P;
        pair_setup<L, VT>(P, k, m_rs, m_rcp, m_eb, m_base, m_amp, shift, a);
        int c = 0;
        for (; P.total - c > 64; c += 128) {
            const int e0 = c + lane, e1 = e0 + 64;  // e0 < total
            float2 v0, v1;
            int w0, w1;
            pair_entry<L, VT>(P, e0, v0, w0);
            if (e1 < P.total) pair_entry<L, VT>(P, e1, v1, w1);
            lds_add(acc, w0, v0, P.sa);
            if (e1 < P.total) lds_add(acc, w1, v1, P.sa);
        }
        if (c + lane < P.total) {
            float2 v0;
            int w0;
            pair_entry<L, VT>(P, c + lane, v0, w0);
            lds_add(acc, w0, v0, P.sa);
        }
    }
}

// One fixed-point word of the tile as FP32 (re, im), scaled by 2^e2 (e2 = -shift).  In FP32: the
// integer is rounded once to 24 bits and then scaled exactly, which is the same rounding as
// scaling in FP64 and converting (for results above the FP32 normal range's floor).
__device__ inline float2 fixed_value(unsigned long long w, int e2)
{
    const int re = (int)(unsigned)w, im = (int)(unsigned)(w >> 32);
    return make_float2(ldexpf((float)re, e2), ldexpf((float)im, e2));
}

// One 2D inverse Haar step for one output of a quadruple, without the factor 1/2: the output at row
// parity a, column parity b of the next finer level, for inputs that carry the halvings of every
// level they still pass through (a level-l coefficient pre-scaled by 2^-l).  Scaling by powers of
// two is exact, so this gives bit for bit the values of the halving step applied level by level,
// with the same additions in the same order as the in-LDS inverse.
__device__ inline float2 haar_up(float2 s, float2 h, float2 v, float2 d, int a, int b)
{
    const float hr = b ? -h.x : h.x, hi = b ? -h.y : h.y;
    const float vr = a ? -v.x : v.x, vi = a ? -v.y : v.y;
    const float dr = (a ^ b) ? -d.x : d.x, di = (a ^ b) ? -d.y : d.y;
    return make_float2(s.x + hr + vr + dr, s.y + hi + vi + di);
}

// Inverse Haar of the tile from its fixed-point words.  The coarse quarter of every block (levels
// >= 2 and the scaling band, its top-left B/2 x B/2 corner) is turned into FP32 (re, im) in place
// and inverted in LDS down to level 1; the finest level, three quarters of the coefficients, goes
// from the fixed-point words through registers straight to the pixels: a thread takes one level-1
// position, i.e. a 2 x 2 pixel quad, and the threads of a wave take consecutive quads of a row, so
// each store instruction writes whole rows of the tile.
template <int L, int NT>
__device__ inline void fixed_inverse_store(unsigned long long *acc, int e2, float2 *out,
                                           int64_t ld, int ty, int tx, int th, int tw)
{
    using S = TileShape<L>;
    constexpr int B = S::B, H1 = B / 2, QT = kT / 2;   // level-1 band extent in a block / tile
    float2 *f = reinterpret_cast<float2 *>(acc);
    auto word = [](int blk, int m, int n) { return (blk / S::TB) * S::ROW + (blk % S::TB) * S::BS + m * B + n; };
    // the coarse quarter in FP32, each coefficient pre-scaled by 2^-l for its level l (l = L for the
    // scaling coefficient, L - floor(log2 max(m, n)) for a detail coefficient at (m, n))
    for (int i = threadIdx.x; i < QT * QT; i += NT) {
        const int m = (i % (H1 * H1)) / H1, n = i % H1, mx = max(m, n);
        const int lev = mx == 0 ? L : L - (31 - __clz(mx));
        const int at = word(i / (H1 * H1), m, n);
        f[at] = fixed_value(acc[at], e2 - lev);
    }
    __syncthreads();
#pragma unroll
    for (int l = L; l >= 2; --l) {
        const int h = B >> l, per = h * h, nq = (kT >> l) * (kT >> l);
        constexpr int MAXQ = ((kT / 4) * (kT / 4) + NT - 1) / NT;
        float2 q[MAXQ][4];
        int at0[MAXQ];
#pragma unroll
        for (int k = 0; k < MAXQ; ++k) {
            const int qi = threadIdx.x + NT * k;
            if (qi < nq) {
                const int blk = qi / per, m = (qi % per) / h, n = qi % h;
                const int s0 = word(blk, m, n);
                at0[k] = word(blk, 2 * m, 2 * n);
                q[k][0] = f[s0];
                q[k][1] = f[s0 + h];
                q[k][2] = f[s0 + h * B];
                q[k][3] = f[s0 + h * B + h];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < MAXQ; ++k) {
            const int qi = threadIdx.x + NT * k;
            if (qi < nq) {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) f[at0[k] + i * B + j] = haar_up(q[k][0], q[k][1], q[k][2], q[k][3], i, j);
            }
        }
        __syncthreads();
    }
    // The pixels are written with non-temporal stores: the hologram is not read again here, and
    // streaming it past the caches keeps the table entries there (65536^2, gamma 0.02: 14.3 -> 12.6 ms).
    const bool wide = ((reinterpret_cast<uintptr_t>(out) | (uintptr_t)ld * sizeof(float2)) & 15) == 0;
    for (int qi = threadIdx.x; qi < QT * QT; qi += NT) {
        const int qm = qi / QT, qn = qi % QT;           // quad row / column in the tile
        const int br = qm / H1, bc = qn / H1, m = qm % H1, n = qn % H1;
        if (br >= (th >> L) || bc >= (tw >> L)) continue;
        const int blk = br * S::TB + bc;
        const float2 S1 = f[word(blk, m, n)];
        const float2 H = fixed_value(acc[word(blk, m, H1 + n)], e2 - 1);
        const float2 V = fixed_value(acc[word(blk, H1 + m, n)], e2 - 1);
        const float2 D = fixed_value(acc[word(blk, H1 + m, H1 + n)], e2 - 1);
        float2 *o = out + ((int64_t)ty * kT + 2 * qm) * ld + (int64_t)tx * kT + 2 * qn;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const float2 p0 = haar_up(S1, H, V, D, i, 0), p1 = haar_up(S1, H, V, D, i, 1);
            if (wide) {
                __builtin_nontemporal_store((v4f){p0.x, p0.y, p1.x, p1.y}, reinterpret_cast<v4f *>(o + i * ld));
            } else {
                __builtin_nontemporal_store((v2f){p0.x, p0.y}, reinterpret_cast<v2f *>(o + i * ld));
                __builtin_nontemporal_store((v2f){p1.x, p1.y}, reinterpret_cast<v2f *>(o + i * ld + 1));
            }
        }
    }
}

// The tile's coefficients from its fixed-point words straight into the window's Mallat layout.
template <int L, int NT>
__device__ inline void fixed_mallat_store(const unsigned long long *acc, int e2, float2 *field,
                                          const TileGeom &g, int ty, int tx, int th, int tw, bool nt,
                                          bool add)
{
    using S = TileShape<L>;
    const int64_t nx = g.nx;
#pragma unroll
    for (int l = 1; l <= L; ++l) {
        const int wf = kT >> l, h = S::B >> l;
        const int hb = th >> l, wb = tw >> l;
#pragma unroll
        for (int band = 1; band <= 3; ++band) {
            const int64_t row0 = (band & 2) ? (g.ny >> l) : 0, col0 = (band & 1) ? (g.nx >> l) : 0;
            for (int i = threadIdx.x; i < wf * wf; i += NT) {
                const int m = i / wf, n = i % wf;
                if (m >= hb || n >= wb) continue;
                const int code = (((band & 2) ? h : 0) + (m & (h - 1))) * S::B + ((band & 1) ? h : 0) + (n & (h - 1));
                put2(field + (row0 + (int64_t)ty * wf + m) * nx + col0 + (int64_t)tx * wf + n,
                     fixed_value(acc[(m / h) * S::ROW + (n / h) * S::BS + code], e2), nt, add);
            }
        }
    }
    constexpr int wf = kT >> L;
    const int hb = th >> L, wb = tw >> L;
    for (int i = threadIdx.x; i < wf * wf; i += NT) {
        const int m = i / wf, n = i % wf;
        if (m >= hb || n >= wb) continue;
        put2(field + ((int64_t)ty * wf + m) * nx + (int64_t)tx * wf + n, fixed_value(acc[m * S::ROW + n * S::BS], e2),
             nt, add);
    }
}

// At L <= 3 the pair walk holds more row values in scalar registers than 8 waves per SIMD leave
// (about 100 SGPRs: 7 waves, i.e. 3 tiles of 8 waves per CU instead of 4); the occupancy hint
// makes the compiler fit them (a few spills to VGPR lanes): 16384^2 FP16 5.53 -> 5.11 ms.  At
// L >= 4 the kernel fits without it.
template <int L, int VT, int MODE>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(L <= 3 ? 8 : 1, 8)))
void tile_kernel(TileArgs a)
{
    using S = TileShape<L>;
    constexpr int NW = kTileThreads / 64;
    // packed fixed-point (re, im) words
    __shared__ unsigned long long acc[S::N];
    const int tile = blockIdx.x;
    int ty, tx;
    tile_of<true>(tile, a.g, ty, tx);
    const int th = min(kT, a.g.ny - ty * kT), tw = min(kT, a.g.nx - tx * kT);
    const int tbh = th >> L, tbw = tw >> L;
    const int sup = a.g.cell / kT;  // the tile's list cell:
    const int lst = ((ty + a.g.lty0) / sup) * a.g.nlx + (tx + a.g.ltx0) / sup;
    const int64_t p0 = a.tile_off[lst], p1 = a.tile_off[lst + 1];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform

    // bound of every coefficient of this tile (its cell's) -> fixed-point scale 2^shift
    for (int i = threadIdx.x; i < S::N; i += kTileThreads) acc[i] = 0;
    const double bound = a.cell_bound[lst];
    __syncthreads();
    int ex;
    (void)frexp(bound * (1.0 + 1e-6) + 1e-300, &ex);  // bound < 2^ex
    const int shift = min(30 - ex, 1000);

    const int64_t gy0 = a.g.oy + (int64_t)ty * kT, gx0 = a.g.ox + (int64_t)tx * kT;
    // Waves take interleaved pairs (wave w: pairs w, w + NW, ...), so the waves of a tile work
    // on neighbouring list positions, i.e. on the same LUT planes.  Each wave gathers the
    // metadata of 64 pairs at once (one pair per lane), then walks them.
    for (int64_t pb = p0 + wave; pb < p1; pb += 64 * NW) {
        const int64_t pk = pb + (int64_t)lane * NW;
        int m_nrows = 0, m_bo = 0, m_nb = 0, m_bc0 = 0, m_bc1 = 0, m_eb = 0, m_dst0 = 0;
        float m_amp = 0.0f;
        if (pk < p1) {
            const wasabi_point pt = a.pts[a.tile_pts[pk]];
            const DepthDesc dd = a.desc[pt.depth];
            const int64_t xg = (int64_t)(pt.x >> L) << L, yg = (int64_t)(pt.y >> L) << L;
            const int obr = (int)((yg - dd.W / 2 - gy0) >> L);  // table block (0,0) in tile blocks
            const int obc = (int)((xg - dd.W / 2 - gx0) >> L);
            const int br0 = max(dd.br0, -obr), br1 = min(dd.br1, tbh - obr);
            const int bc0 = max(dd.bc0, -obc), bc1 = min(dd.bc1, tbw - obc);
            if (br0 < br1 && bc0 < bc1) {
                m_nrows = br1 - br0;
                m_bo = (int)(dd.blkoff_base + (int64_t)br0 * dd.nb);
                m_nb = dd.nb;
                m_bc0 = bc0;
                m_bc1 = bc1;
                m_eb = (int)dd.entry_base;
                // L >= 3: the LDS word of the table's block (0, 0); L <= 2: of the pair's first block
                m_dst0 = S::TB <= 8 ? obr * S::ROW + obc * S::BS : (br0 + obr) * S::ROW + obc * S::BS;
                m_amp = pt.a;
            }
        }
        const int cnt = (int)min((int64_t)64, (p1 - pb + NW - 1) / NW);
        if constexpr (S::TB <= 8) {
            walk_pairs<L, VT>(acc, a, cnt, m_nrows, m_bo, m_nb, m_bc0, m_bc1, m_eb, m_dst0, m_amp, shift);
            continue;
        }
        // software pipeline: the row ranges of the next pair load while this pair's entries run
        int k = 0;
        while (k < cnt && __builtin_amdgcn_readlane(m_nrows, k) == 0) ++k;
        int rstart = 0, rcount = 0;
        if (k < cnt) {
            const int nrows = __builtin_amdgcn_readlane(m_nrows, k);
            if (lane < nrows) {
                const int32_t *r = a.blk_off + __builtin_amdgcn_readlane(m_bo, k) + lane * __builtin_amdgcn_readlane(m_nb, k);
                rstart = r[__builtin_amdgcn_readlane(m_bc0, k)];
                rcount = r[__builtin_amdgcn_readlane(m_bc1, k)] - rstart;
            }
        }
        while (k < cnt) {
            int kn = k + 1;
            while (kn < cnt && __builtin_amdgcn_readlane(m_nrows, kn) == 0) ++kn;
            int nstart = 0, nend = 0;
            if (kn < cnt) {
                const int nrows = __builtin_amdgcn_readlane(m_nrows, kn);
                if (lane < nrows) {
                    const int32_t *r = a.blk_off + __builtin_amdgcn_readlane(m_bo, kn) + lane * __builtin_amdgcn_readlane(m_nb, kn);
                    nstart = r[__builtin_amdgcn_readlane(m_bc0, kn)];
                    nend = r[__builtin_amdgcn_readlane(m_bc1, kn)];
                }
            }
            const float amp = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m_amp), k));
            add_pair<L, VT>(acc, a.values, a.keys, __builtin_amdgcn_readlane(m_eb, k),
                            __builtin_amdgcn_readlane(m_dst0, k), __builtin_amdgcn_readlane(m_nrows, k),
                            ldexp((double)amp, shift), rstart, rcount);
            rstart = nstart;
            rcount = nend - nstart;
            k = kn;
        }
    }
    __syncthreads();

    const int e2 = -shift;  // the words hold value * 2^shift
    if constexpr (MODE == MODE_PSI)
        fixed_mallat_store<L, kTileThreads>(acc, e2, a.out, a.g, ty, tx, th, tw, a.stream_psi != 0,
                                            a.accumulate != 0);
    else
        fixed_inverse_store<L, kTileThreads>(acc, e2, a.out, a.ld, ty, tx, th, tw);
}

// Dense-layout superposition.  Wave w of the tile's 8 waves owns the 512 coefficients
// [512 w, 512 w + 512) of the tile (block-major order, i.e. block row w for L = 3) and keeps them in
// FP32 registers, lane = code: for every point of the tile (in list order) it reads the table
// blocks that fall on its coefficients -- a contiguous run per table block row -- and does
// acc += a_j * c.  No LDS traffic, no atomics; every coefficient is summed in list order.
constexpr int kDenseThreads = 512;
constexpr int kPaceSpin = 20000;       // ~ a few ms of polling at most, then pacing is dropped
constexpr int kPaceMaxPlanes = 4096;  // plane bounds live in the tile's LDS staging buffer
constexpr int kPaceCounters = 64;     // counter words per plane

template <int L, int VT, int MODE>
__global__ __launch_bounds__(kDenseThreads) __attribute__((amdgpu_waves_per_eu(8, 8)))
void dense_tile_kernel(TileArgs a)
{
    using S = TileShape<L>;
    constexpr int BB = S::B * S::B;
    constexpr int NW = kDenseThreads / 64;
    constexpr int PER = kT * kT / kDenseThreads;  // coefficients per lane (8)
    __shared__ float sbuf[2 * S::N];
    const int tile = blockIdx.x;
    int ty, tx;
    tile_of_cells(tile, a.g, ty, tx);
    const int th = min(kT, a.g.ny - ty * kT), tw = min(kT, a.g.nx - tx * kT);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sup = a.g.cell / kT;  // the tile's list cell:
    const int lst = ((ty + a.g.lty0) / sup) * a.g.nlx + (tx + a.g.ltx0) / sup;
    const int64_t p0 = a.tile_off[lst], p1 = a.tile_off[lst + 1];
    const int64_t gy0 = a.g.oy + (int64_t)ty * kT, gx0 = a.g.ox + (int64_t)tx * kT;

    // The lane's coefficient i (of PER = 8), as an index c in the tile's block-major order: tile
    // block b = c / BB (block row b / TB, column b % TB), code c % BB.  For L >= 3 a lane holds
    // coefficient i = k E + e as 512 w + 64 E k + E lane + e, so that one 16-byte load per k
    // fetches the lane's E consecutive codes; for L < 3, c = 512 w + 64 i + lane.  Recomputed where
    // needed rather than held in registers.
    constexpr int E = BB >= 64 ? Wide<VT>::E : 1;
    auto coef_of = [&](int i) {
        return BB >= 64 ? wave * 512 + 64 * E * (i / E) + E * lane + i % E : wave * 512 + i * 64 + lane;
    };
    auto tbr_of = [&](int i) { return (coef_of(i) / BB) / S::TB; };
    auto tbc_of = [&](int i) { return (coef_of(i) / BB) % S::TB; };
    auto code_of = [&](int i) { return coef_of(i) % BB; };
    float are[PER], aim[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) are[i] = aim[i] = 0.0f;

    if (BB >= 64) {
        // For L >= 3 the wave's coefficients lie in one tile block row (tr) and tile block columns
        // tbc_of(i); per pair only one table block row (tr - obr) is involved.  Lane k resolves pair k
        // of each 64-pair batch up to the address of its first coefficient (one parallel pass over
        // the dependent loads), then the wave walks the pairs.
        const int tr = tbr_of(0);
        auto run = [&](int64_t q0, int64_t q1) {
            for (int64_t pb = q0; pb < q1; pb += 64) {
                const int64_t pk = pb + lane;
                int m_clo = 0, m_chi = 0;  // tile block columns [clo, chi) the pair covers
                int m_blo = 0, m_bhi = 0;  // address of tile block column 0 (64-bit, split)
                float m_amp = 0.0f;
                if (pk < q1) {
                    const wasabi_point pt = a.pts[a.tile_pts[pk]];
                    const DepthDesc dd = a.desc[pt.depth];
                    const int64_t xg = (int64_t)(pt.x >> L) << L, yg = (int64_t)(pt.y >> L) << L;
                    const int obr = (int)((yg - dd.W / 2 - gy0) >> L);
                    const int obc = (int)((xg - dd.W / 2 - gx0) >> L);
                    const int br = tr - obr;
                    if (br >= dd.br0 && br < dd.br1) {
                        const DenseRow row = a.dense_rows[dd.rows_base + br];
                        m_clo = max(row.lo + obc, 0);
                        m_chi = min(row.hi + obc, S::TB);
                        const int64_t b0 = dd.dense_base + row.off - (int64_t)(row.lo + obc) * BB;
                        m_blo = (int)(b0 & 0xffffffff);
                        m_bhi = (int)(b0 >> 32);
                        m_amp = pt.a;
                    }
                }
                const int cnt = (int)min((int64_t)64, q1 - pb);
                // one 16-byte load per E coefficients of a lane; a block the pair does not cover
                // reads the zero values instead, so the loads and FMAs need no branches
                const int wofs = (wave * 512) % (BB * S::TB);  // the wave's first coefficient in its row
                for (int k = 0; k < cnt; ++k) {
                    const int clo = __builtin_amdgcn_readlane(m_clo, k), chi = __builtin_amdgcn_readlane(m_chi, k);
                    if (chi <= clo) continue;
                    const int64_t b0 = ((int64_t)__builtin_amdgcn_readlane(m_bhi, k) << 32) | (uint32_t)__builtin_amdgcn_readlane(m_blo, k);
                    const float amp = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m_amp), k));
                    float2 v[PER];
#pragma unroll
                    for (int j = 0; j < PER / E; ++j) {
                        const int tc = tbc_of(j * E);
                        const int64_t rel = 64 * E * j + E * lane;
                        const int64_t at = (tc >= clo && tc < chi) ? b0 + wofs + rel : a.dense_zero + rel;
                        load_wide<VT>(a.dense, at, v + j * E);
                    }
#pragma unroll
                    for (int i = 0; i < PER; ++i) {
                        are[i] = fmaf(amp, v[i].x, are[i]);
                        aim[i] = fmaf(amp, v[i].y, aim[i]);
                    }
                }
            }
        };
        if (a.plane_done == nullptr) {
            run(p0, p1);
        } else {
            // Plane pacing.  The tile's list is in plane order; all resident tiles walk the planes
            // together (a tile starts plane d only after every tile finished plane d - slack), so
            // the table bands being read at any moment stay in L2.  Every wait is bounded: after
            // kPaceSpin polls a tile stops waiting for good, so progress never depends on it.
            int *bnd = (int *)sbuf;  // plane d owns list positions [bnd[d], bnd[d + 1])
            const int nd = a.n_tables;
            for (int d = threadIdx.x; d <= nd; d += kDenseThreads) bnd[d] = 0;
            __syncthreads();
            for (int64_t p = p0 + threadIdx.x; p < p1; p += kDenseThreads) {
                const int d = a.pts[a.tile_pts[p]].depth;
                const int dn = (p + 1 < p1) ? a.pts[a.tile_pts[p + 1]].depth : nd;
                for (int e = d + 1; e <= dn; ++e) bnd[e] = (int)(p + 1 - p0);  // ends of planes d..dn-1
            }
            __syncthreads();
            // planes before the first one present start at 0; fill the gaps forward
            if (threadIdx.x == 0) {
                int last = 0;
                for (int d = 0; d <= nd; ++d) {
                    if (bnd[d] < last) bnd[d] = last;
                    last = bnd[d];
                }
            }
            __syncthreads();
            // plane d's counter is spread over kPaceCounters words (tile t counts into word t % 64),
            // so the 64 lanes of wave 0 poll them in parallel and no word sees more than a few adds
            bool pacing = true;
            const int ntiles = a.g.ntx * a.g.nty;
            const int my_word = tile % kPaceCounters;
            const int want = ntiles / kPaceCounters + (lane < ntiles % kPaceCounters ? 1 : 0);
            __shared__ int s_go;
            // A plane without points in the tile's list needs neither a wait nor a barrier: it is
            // finished as soon as the planes before it are, and only its counter moves (with
            // hundreds of planes and a tile's points in a few dozen of them, a wait at every plane
            // costs a memory round trip each).
            for (int d = 0; d < nd; ++d) {
                const int64_t q0 = p0 + bnd[d], q1 = p0 + bnd[d + 1];
                if (q1 > q0) {
                    if (pacing && d >= a.pace_slack) {
                        if (wave == 0) {
                            const int *w = a.plane_done + (int64_t)(d - a.pace_slack) * kPaceCounters + lane;
                            int it = 0;
                            while (it < kPaceSpin) {
                                const bool ok = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= want;
                                if (__ballot(!ok) == 0) break;
                                __builtin_amdgcn_s_sleep(2);
                                ++it;
                            }
                            if (lane == 0) s_go = it < kPaceSpin;
                        }
                        __syncthreads();
                        pacing = s_go != 0;
                    }
                    run(q0, q1);
                    __syncthreads();
                }
                if (threadIdx.x == 0)
                    __hip_atomic_fetch_add(a.plane_done + (int64_t)d * kPaceCounters + my_word, 1,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
        }
    } else {
        for (int64_t pb = p0; pb < p1; pb += 64) {
            const int64_t pk = pb + lane;
            int m_d = 0, m_obr = 0, m_obc = 0;
            float m_amp = 0.0f;
            if (pk < p1) {
                const wasabi_point pt = a.pts[a.tile_pts[pk]];
                const int W = a.desc[pt.depth].W;
                const int64_t xg = (int64_t)(pt.x >> L) << L, yg = (int64_t)(pt.y >> L) << L;
                m_d = pt.depth;
                m_obr = (int)((yg - W / 2 - gy0) >> L);
                m_obc = (int)((xg - W / 2 - gx0) >> L);
                m_amp = pt.a;
            }
            const int cnt = (int)min((int64_t)64, p1 - pb);
            for (int k = 0; k < cnt; ++k) {
                const int d = __builtin_amdgcn_readlane(m_d, k);
                const int obr = __builtin_amdgcn_readlane(m_obr, k);
                const int obc = __builtin_amdgcn_readlane(m_obc, k);
                const float amp = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m_amp), k));
                const DepthDesc &dd = a.desc[d];
                const int64_t base = dd.dense_base;
                const DenseRow *rows = a.dense_rows + dd.rows_base;
#pragma unroll
                for (int i = 0; i < PER; ++i) {
                    const int br = tbr_of(i) - obr, bc = tbc_of(i) - obc;
                    if (br < dd.br0 || br >= dd.br1) continue;
                    const DenseRow row = rows[br];
                    if (bc < row.lo || bc >= row.hi) continue;
                    const float2 v = load_value<VT>(a.dense, base + row.off + (int64_t)(bc - row.lo) * BB + code_of(i));
                    are[i] = fmaf(amp, v.x, are[i]);
                    aim[i] = fmaf(amp, v.y, aim[i]);
                }
            }
        }
    }

    // registers -> LDS (tile block layout) -> inverse or Mallat output
    float *sre = sbuf, *sim = sbuf + S::N;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int at = tbr_of(i) * S::ROW + tbc_of(i) * S::BS + code_of(i);
        sre[at] = are[i];
        sim[at] = aim[i];
    }
    __syncthreads();
    if (MODE == MODE_PSI) {
        tile_mallat_io<L, false, kDenseThreads>(sre, sim, a.out, a.g, ty, tx, th, tw, a.accumulate != 0);
    } else {
        tile_inverse_and_store<L, kDenseThreads, true>(sre, sim, a.out, a.ld, ty, tx, th, tw);
    }
    (void)NW;
}

template <int L>
__global__ __launch_bounds__(kThreads) void idwt_kernel(TileArgs a)
{
    using S = TileShape<L>;
    __shared__ float sre[S::N];
    __shared__ float sim[S::N];
    const int tile = blockIdx.x;
    int ty, tx;
    tile_of(tile, a.g, ty, tx);
    const int th = min(kT, a.g.ny - ty * kT), tw = min(kT, a.g.nx - tx * kT);
    tile_mallat_load<L, kThreads>(sre, sim, a.in, a.g, ty, tx, th, tw);
    __syncthreads();
    tile_inverse_and_store<L, kThreads>(sre, sim, a.out, a.ld, ty, tx, th, tw);
}

// ---- host side ------------------------------------------------------------------------------
TileGeom make_geom(int64_t ox, int64_t oy, int32_t nx, int32_t ny)
{
    TileGeom g;
    g.ox = ox;
    g.oy = oy;
    g.nx = nx;
    g.ny = ny;
    g.ntx = (nx + kT - 1) / kT;
    g.nty = (ny + kT - 1) / kT;
    g.cell = kT;
    g.nlx = g.ntx;
    g.nly = g.nty;
    g.ltx0 = g.lty0 = 0;
    return g;
}

// Point lists per tile while there are at most kMaxLdsTiles tiles; beyond that per square of
// 2 x 2 or 4 x 4 tiles (the smallest that gives at most kMaxLdsTiles lists, 4 x 4 at most).  A
// tile then walks its cell's list and skips the points that miss it: each point goes to far fewer
// lists (binning is per (point, list) pair) at the price of a few more pairs per tile.
void choose_lists(TileGeom &g)
{
    int sup = 1;
    while (sup < 4 && (int64_t)((g.ntx + sup - 1) / sup) * ((g.nty + sup - 1) / sup) > kMaxLdsTiles) sup *= 2;
    g.cell = kT * sup;
    g.nlx = (g.ntx + sup - 1) / sup;
    g.nly = (g.nty + sup - 1) / sup;
}

int check_window(int L, int64_t ox, int64_t oy, int32_t nx, int32_t ny)
{
    const int B = 1 << L;
    if (nx < B || ny < B || nx % B || ny % B)
        return fail(CGH_EINVAL, "window %d x %d must be a positive multiple of 2^L = %d", nx, ny, B);
    if (ox % B || oy % B) return fail(CGH_EINVAL, "window origin must be a multiple of 2^L = %d", B);
    const int64_t lim = INT64_C(1) << 40;
    if (ox < -lim || oy < -lim || ox > lim || oy > lim) return fail(CGH_EINVAL, "window origin out of range");
    return CGH_OK;
}

}  // namespace

// Exclusive scan of `count` int32 values into int64 offsets (count + 1 values) on stream s.
// Exclusive scan of count int32 counts into count + 1 int64 offsets; short arrays (up to 16384) in
// one workgroup, which also writes the offsets into `copy` when it is not NULL.
int scan_counts_copy(const int32_t *counts, int64_t count, int64_t *off, Scratch &sc, hipStream_t s,
                     unsigned long long *copy)
{
    if (count <= 16384) {
        hipLaunchKernelGGL(scan_small_kernel, dim3(1), dim3(1024), 0, s, counts, count, off, copy);
        CGH_CHECK_LAUNCH("scan_small_kernel");
        return CGH_OK;
    }
    if (copy) return fail(CGH_EINVAL, "scan copy needs at most 16384 counts");
    const int64_t nblk = (count + 1023) / 1024;
    int64_t *bsum;
    int rc = sc.alloc((void **)&bsum, sizeof(int64_t) * nblk);
    if (rc) return rc;
    hipLaunchKernelGGL(scan_local_kernel, dim3((unsigned)nblk), dim3(1024), 0, s, counts, count, off, bsum);
    CGH_CHECK_LAUNCH("scan_local_kernel");
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, s, bsum, nblk, off + count);
    CGH_CHECK_LAUNCH("scan_sums_kernel");
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, off, count, bsum);
    CGH_CHECK_LAUNCH("scan_add_kernel");
    return CGH_OK;
}

int scan_counts(const int32_t *counts, int64_t count, int64_t *off, Scratch &sc, hipStream_t s)
{
    return scan_counts_copy(counts, count, off, sc, s, nullptr);
}

namespace {

// Bins of the plane sort: (plane, 64-row band of the point's y) pairs plus one for invalid points.
int sort_bands(const wasabi_lut *lut, const TileGeom &g)
{
    const int nd = lut->n_tables;
    int nyb = (int)std::min<int64_t>(((int64_t)g.ny + 2 * lut->max_span_px + 63) / 64, 4096);
    if ((int64_t)nyb * nd + 1 > (INT64_C(1) << 26)) nyb = std::max(1, (1 << 26) / nd - 1);
    // The bands only order a plane's points for locality (points beyond the last band join it), so
    // a few fewer of them are harmless; when that keeps the bin count within a power of two, the
    // radix sort may need a pass less (64 planes x 64 bands + 1 = 4097 bins -> 63 bands, 12 bits).
    for (int b = 8; b <= 26; ++b) {
        const int64_t cap = INT64_C(1) << b;
        if ((int64_t)nyb * nd + 1 > cap) {
            const int64_t fit = (cap - 1) / nd;
            if (fit >= 1 && fit >= nyb - nyb / 16) {
                nyb = (int)fit;
                break;
            }
        }
    }
    return nyb;
}

// (list cell, point) pairs the lists can hold: every point meets at most per_point cells.
int64_t pair_bound(const wasabi_lut *lut, int64_t n, const TileGeom &g)
{
    const int64_t nlists = (int64_t)g.nlx * g.nly;
    const int64_t per_side = (lut->max_span_px + g.cell - 1) / g.cell + 1;
    const int64_t per_point = std::min<int64_t>(per_side * per_side, nlists);
    return std::max<int64_t>(n * per_point, 1);
}

bool use_matrix_path(int64_t n, int64_t ntiles)
{
    const int64_t nwg = (n + chunk_pts(n) - 1) / chunk_pts(n);
    return n > 0 && ntiles <= kMaxLdsTiles && nwg * ntiles <= (INT64_C(1) << 24);
}

// Bits needed for the keys 0 .. count - 1.
inline int key_bits(int64_t count)
{
    int b = 1;
    while ((INT64_C(1) << b) < count) ++b;
    return b;
}

// Passes, digit bits and blocks of a radix sort of at most n_max items with keys of kbits bits.
// Blocks take 4096 items; for short arrays fewer, larger blocks keep the digit matrix within one
// workgroup's scan (16384 entries).
struct RadixPlan {
    int passes, bits, nblk;
    int64_t per;
};

inline RadixPlan radix_plan(int64_t n_max, int kbits)
{
    RadixPlan p;
    p.passes = std::max(1, (kbits + kSortMaxBits - 1) / kSortMaxBits);
    p.bits = (kbits + p.passes - 1) / p.passes;
    const int64_t D = INT64_C(1) << p.bits, n = std::max<int64_t>(n_max, 1);
    int64_t nblk = (n + 4095) / 4096;
    if (n <= 65536) nblk = std::max<int64_t>(1, std::min<int64_t>(nblk, 16384 / D));
    p.per = (n + nblk - 1) / nblk;
    p.nblk = (int)((n + p.per - 1) / p.per);
    return p;
}

inline int64_t scratch_round(int64_t b) { return std::max<int64_t>((b + 255) / 256 * 256, 256); }

// Scratch bytes a multi-block exclusive scan of `count` counts takes (none up to 16384).
inline int64_t scan_scratch(int64_t count) { return count <= 16384 ? 0 : scratch_round(8 * ((count + 1023) / 1024)); }

// Scratch bytes of radix_sort for n_max items of `item` bytes.
inline int64_t radix_scratch(int64_t n_max, int kbits, int64_t item)
{
    if (n_max <= 0) return 0;
    const RadixPlan p = radix_plan(n_max, kbits);
    const int64_t cells = (INT64_C(1) << p.bits) * p.nblk;
    return scratch_round(4 * cells) + scratch_round(8 * (cells + 1)) + scan_scratch(cells) +
           std::min(p.passes - 1, 2) * scratch_round(item * n_max);
}

// Stable LSD radix sort of n items (n_max on the host; n_dev, when not NULL, the device-resident
// count, at most n_max) by key() into `out`, or for pairs their low 32 bits into `out_low`.
template <class K>
int radix_sort(const typename K::T *in, int64_t n_max, const int64_t *n_dev, K key, int kbits,
               typename K::T *out, int32_t *out_low, Scratch &sc, hipStream_t s)
{
    using T = typename K::T;
    if (n_max <= 0) return CGH_OK;
    const RadixPlan P = radix_plan(n_max, kbits);
    const int D = 1 << P.bits;
    const int64_t cells = (int64_t)D * P.nblk;
    int32_t *mat;
    int64_t *moff;
    T *tmp[2] = {nullptr, nullptr};
    int rc;
    if ((rc = sc.alloc((void **)&mat, sizeof(int32_t) * cells))) return rc;
    if ((rc = sc.alloc((void **)&moff, sizeof(int64_t) * (cells + 1)))) return rc;
    for (int i = 0; i < std::min(P.passes - 1, 2); ++i)
        if ((rc = sc.alloc((void **)&tmp[i], sizeof(T) * n_max))) return rc;
    const T *src = in;
    for (int p = 0; p < P.passes; ++p) {
        const bool last = p == P.passes - 1;
        T *dst = last ? out : tmp[p % 2];
        hipLaunchKernelGGL(radix_count_kernel<K>, dim3(P.nblk), dim3(kSortThreads), sizeof(int) * D, s, src,
                           n_max, n_dev, key, p * P.bits, P.bits, P.per, P.nblk, mat);
        CGH_CHECK_LAUNCH("radix_count_kernel");
        if ((rc = scan_counts(mat, cells, moff, sc, s))) return rc;
        hipLaunchKernelGGL(radix_scatter_kernel<K>, dim3(P.nblk), dim3(kSortThreads),
                           (sizeof(int) + 4 * sizeof(unsigned short)) * D, s, src, n_max, n_dev, key,
                           p * P.bits, P.bits, P.per, P.nblk, moff, dst, last ? out_low : nullptr);
        CGH_CHECK_LAUNCH("radix_scatter_kernel");
        src = dst;
    }
    return CGH_OK;
}

// Plane-sort the points and build the per-tile point lists; results live in `sc`.  Every step
// is deterministic except the list fill of the sparse layout beyond kMaxLdsTiles cells (atomic
// cursors), whose fixed-point sums do not depend on the list order.
int bin_points(const wasabi_lut *lut, const wasabi_point *pts, int64_t n, const TileGeom &g,
               Scratch &sc, hipStream_t s, const wasabi_point **sorted_out,
               int64_t **tile_off_out, int32_t **tile_pts_out, double **bound_out, bool *ordered_out)
{
    const int64_t ntiles = (int64_t)g.nlx * g.nly;  // lists
    const int64_t bound = pair_bound(lut, n, g);
    const int nd = lut->n_tables, L = lut->L;
    SortKey key;
    key.n_tables = nd;
    key.y0 = g.oy - lut->max_span_px;
    key.nyb = sort_bands(lut, g);
    const int64_t nbins = (int64_t)nd * key.nyb + 1;
    int32_t *counts;
    int64_t *off;
    int32_t *list;
    wasabi_point *sorted;
    int rc;
    if ((rc = sc.alloc((void **)&counts, sizeof(int32_t) * ntiles))) return rc;
    if ((rc = sc.alloc((void **)&off, sizeof(int64_t) * (ntiles + 1)))) return rc;
    if ((rc = sc.alloc((void **)&list, sizeof(int32_t) * bound))) return rc;
    if ((rc = sc.alloc((void **)&sorted, sizeof(wasabi_point) * std::max<int64_t>(n, 1)))) return rc;
    ProfScope prof("bin", s);
    // plane sort: stable, by (plane, row band)
    PointKey pk;
    pk.k = key;
    if ((rc = radix_sort(pts, n, nullptr, pk, key_bits(nbins), sorted, nullptr, sc, s))) return rc;
    // tile lists over the sorted points
    const int64_t nwg = (n + chunk_pts(n) - 1) / chunk_pts(n);
    const unsigned pblocks = (unsigned)((n + 255) / 256);
    *ordered_out = false;
    if (use_matrix_path(n, ntiles)) {
        *ordered_out = true;
        int32_t *mat;
        int64_t *moff;
        if ((rc = sc.alloc((void **)&mat, sizeof(int32_t) * nwg * ntiles))) return rc;
        if ((rc = sc.alloc((void **)&moff, sizeof(int64_t) * (nwg * ntiles + 1)))) return rc;
        hipLaunchKernelGGL(bin_count_matrix_kernel, dim3((unsigned)nwg), dim3(kChunk), 0, s, sorted, n, lut->desc, nd, L, g, (int)nwg, chunk_pts(n), mat);
        CGH_CHECK_LAUNCH("bin_count_matrix_kernel");
        if ((rc = scan_counts(mat, nwg * ntiles, moff, sc, s))) return rc;
        hipLaunchKernelGGL(gather_tile_off_kernel, dim3((unsigned)((ntiles + 256) / 256)), dim3(256), 0, s, moff, ntiles, (int)nwg, off);
        CGH_CHECK_LAUNCH("gather_tile_off_kernel");
        hipLaunchKernelGGL(bin_fill_matrix_kernel, dim3((unsigned)nwg), dim3(kChunk), 0, s, sorted, n, lut->desc, nd, L, g, (int)nwg, chunk_pts(n), moff, list);
        CGH_CHECK_LAUNCH("bin_fill_matrix_kernel");
    } else {
        if ((rc = zero_words(counts, ntiles, s))) return rc;
        const bool lds_tiles = ntiles <= kMaxLdsTiles;
        if (n > 0) {
            if (lds_tiles)
                hipLaunchKernelGGL(bin_count_kernel<true>, dim3(pblocks), dim3(256), 0, s, sorted, n, lut->desc, nd, L, g, counts);
            else
                hipLaunchKernelGGL(bin_count_kernel<false>, dim3(pblocks), dim3(256), 0, s, sorted, n, lut->desc, nd, L, g, counts);
            CGH_CHECK_LAUNCH("bin_count_kernel");
        }
        if ((rc = scan_counts(counts, ntiles, off, sc, s))) return rc;
        if (n > 0 && lut->dense) {
            // the dense kernel sums in list order: the lists keep the sorted order of the points
            if (bound > INT32_MAX) return fail(CGH_EINVAL, "more than 2^31 - 1 (list cell, point) pairs");
            int32_t *pc;
            int64_t *poff;
            unsigned long long *pairs;
            if ((rc = sc.alloc((void **)&pc, sizeof(int32_t) * n))) return rc;
            if ((rc = sc.alloc((void **)&poff, sizeof(int64_t) * (n + 1)))) return rc;
            if ((rc = sc.alloc((void **)&pairs, sizeof(unsigned long long) * bound))) return rc;
            hipLaunchKernelGGL(point_cells_kernel, dim3(pblocks), dim3(256), 0, s, sorted, n, lut->desc, nd, L, g, pc);
            CGH_CHECK_LAUNCH("point_cells_kernel");
            if ((rc = scan_counts(pc, n, poff, sc, s))) return rc;
            hipLaunchKernelGGL(pair_fill_kernel, dim3(pblocks), dim3(256), 0, s, sorted, n, lut->desc, nd, L, g, poff, pairs);
            CGH_CHECK_LAUNCH("pair_fill_kernel");
            if ((rc = radix_sort(pairs, bound, poff + n, PairKey(), key_bits(ntiles), (unsigned long long *)nullptr,
                                 list, sc, s)))
                return rc;
            *ordered_out = true;
        } else if (n > 0) {
            unsigned long long *cursor;
            if ((rc = sc.alloc((void **)&cursor, sizeof(unsigned long long) * ntiles))) return rc;
            CGH_TRY_HIP(hipMemcpyAsync(cursor, off, sizeof(int64_t) * ntiles, hipMemcpyDeviceToDevice, s));
            if (lds_tiles)
                hipLaunchKernelGGL(bin_fill_kernel<true>, dim3(pblocks), dim3(256), 0, s, sorted, n, lut->desc, nd, L, g, cursor, list);
            else
                hipLaunchKernelGGL(bin_fill_kernel<false>, dim3(pblocks), dim3(256), 0, s, sorted, n, lut->desc, nd, L, g, cursor, list);
            CGH_CHECK_LAUNCH("bin_fill_kernel");
        }
    }
    double *cbound;
    if ((rc = sc.alloc((void **)&cbound, sizeof(double) * ntiles))) return rc;
    hipLaunchKernelGGL(cell_bound_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, sorted, list, off, lut->desc, cbound);
    CGH_CHECK_LAUNCH("cell_bound_kernel");
    *sorted_out = sorted;
    *tile_off_out = off;
    *tile_pts_out = list;
    *bound_out = cbound;
    return CGH_OK;
}

// LDS a dense FP32 workgroup reserves when the tiles are not paced, so that at most two tiles share
// a CU (four fit otherwise).  Without pacing the resident tiles cover a region of the grid that
// grows with their number, and so does the table data they read at once; with FP32 values that
// data overflows the L2s.  65536^2, 40 dB selectivity: four tiles per CU 122.7 ms, three 105.5 ms,
// two 96.4 ms, one 121.9 ms.  FP16 values (half the bytes) run best with four (49.8, 53.6, 67.1 ms
// with four, three, two), so they keep the default.
constexpr size_t kDenseF32TileLds = 62 * 1024;

template <int L, int MODE>
void launch_dense_l(int vt, const TileArgs &a, unsigned grid, hipStream_t s)
{
    constexpr size_t stat = sizeof(float) * 2 * TileShape<L>::N + sizeof(int);  // the kernel's own LDS
    const size_t pad = a.plane_done == nullptr && stat < kDenseF32TileLds ? kDenseF32TileLds - stat : 0;
    if (vt == CGH_F32) hipLaunchKernelGGL((dense_tile_kernel<L, CGH_F32, MODE>), dim3(grid), dim3(kDenseThreads), pad, s, a);
    else if (vt == CGH_F16) hipLaunchKernelGGL((dense_tile_kernel<L, CGH_F16, MODE>), dim3(grid), dim3(kDenseThreads), 0, s, a);
    else hipLaunchKernelGGL((dense_tile_kernel<L, CGH_BF16, MODE>), dim3(grid), dim3(kDenseThreads), 0, s, a);
}

template <int L, int MODE>
void launch_tile_l(int vt, const TileArgs &a, unsigned grid, hipStream_t s)
{
    if (a.dense) {
        launch_dense_l<L, MODE>(vt, a, grid, s);
        return;
    }
    if (vt == CGH_F32) hipLaunchKernelGGL((tile_kernel<L, CGH_F32, MODE>), dim3(grid), dim3(kTileThreads), 0, s, a);
    else if (vt == CGH_F16) hipLaunchKernelGGL((tile_kernel<L, CGH_F16, MODE>), dim3(grid), dim3(kTileThreads), 0, s, a);
    else hipLaunchKernelGGL((tile_kernel<L, CGH_BF16, MODE>), dim3(grid), dim3(kTileThreads), 0, s, a);
}

template <int MODE>
int launch_tile(int L, int vt, const TileArgs &a, hipStream_t s)
{
    const int64_t ntiles = (int64_t)a.g.ntx * a.g.nty;
    if (ntiles > INT32_MAX) return fail(CGH_EINVAL, "too many tiles");
    const unsigned grid = (unsigned)ntiles;
    ProfScope prof(MODE == MODE_PSI ? "tile_superpose" : "tile_fused", s);
    switch (L) {
    case 1: launch_tile_l<1, MODE>(vt, a, grid, s); break;
    case 2: launch_tile_l<2, MODE>(vt, a, grid, s); break;
    case 3: launch_tile_l<3, MODE>(vt, a, grid, s); break;
    case 4: launch_tile_l<4, MODE>(vt, a, grid, s); break;
    case 5: launch_tile_l<5, MODE>(vt, a, grid, s); break;
    default: launch_tile_l<6, MODE>(vt, a, grid, s); break;
    }
    CGH_CHECK_LAUNCH("tile_kernel");
    return CGH_OK;
}

// The superposition writes a Mallat field larger than the 256 MiB last-level cache (the Infinity
// Cache) with non-temporal stores.  The field cannot stay cached until the inverse reads it, and
// written through the cache its dirty lines are flushed while the inverse runs (65536^2 in
// 8192^2 sub-holograms: inverse 15.4 -> 14.1 ms, procedure 31.7 -> 30.6 ms).  A smaller field is
// left in the cache, from which the inverse then reads it.  Non-temporal loads in the inverse
// were tried as well and gave nothing.
bool streams_past_cache(int32_t nx, int32_t ny)
{
    return (int64_t)nx * ny * (int64_t)sizeof(float2) > (INT64_C(256) << 20);
}

TileArgs make_args(const wasabi_lut *lut, const wasabi_point *pts, const int64_t *tile_off,
                   const int32_t *tile_pts, const TileGeom &g, float2 *out, int64_t ld)
{
    TileArgs a;
    a.desc = lut ? lut->desc : nullptr;
    a.blk_off = lut ? lut->blk_off : nullptr;
    a.values = lut ? lut->values : nullptr;
    a.keys = lut ? lut->keys : nullptr;
    a.wkeys = lut ? lut->wkeys : nullptr;
    a.pts = pts;
    a.tile_off = tile_off;
    a.tile_pts = tile_pts;
    a.cell_bound = nullptr;
    a.g = g;
    a.in = nullptr;
    a.out = out;
    a.ld = ld;
    a.dense = lut ? lut->dense_values : nullptr;
    a.dense_zero = lut ? lut->dense_zero : 0;
    a.dense_rows = lut ? lut->dense_rows : nullptr;
    a.n_tables = lut ? lut->n_tables : 0;
    a.plane_done = nullptr;
    a.pace_slack = 5;
    a.stream_psi = 0;
    a.accumulate = 0;
    return a;
}

// Workgroups of the dense kernel that fit the device at once (0 if unknown).
template <int L, int VT, int MODE>
int64_t capacity_of()
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dense_tile_kernel<L, VT, MODE>, kDenseThreads, 0) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return (int64_t)per_cu * cus;
}

int64_t resident_capacity(int L, int vt, int mode)
{
    static std::mutex mu;
    static int64_t cache[7][3][2] = {};
    static bool known[7][3][2] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (known[L][vt][mode]) return cache[L][vt][mode];
    int64_t c = 0;
#define CGH_CAP(LL)                                                                                   \
    if (L == LL) {                                                                                    \
        if (vt == CGH_F32) c = mode ? capacity_of<LL, CGH_F32, 1>() : capacity_of<LL, CGH_F32, 0>();    \
        else if (vt == CGH_F16) c = mode ? capacity_of<LL, CGH_F16, 1>() : capacity_of<LL, CGH_F16, 0>(); \
        else c = mode ? capacity_of<LL, CGH_BF16, 1>() : capacity_of<LL, CGH_BF16, 0>();                \
    }
    CGH_CAP(3) CGH_CAP(4) CGH_CAP(5) CGH_CAP(6)
#undef CGH_CAP
    (void)hipGetLastError();
    cache[L][vt][mode] = c;
    known[L][vt][mode] = true;
    return c;
}

// Points binned for a window: the plane-sorted points, the per-cell point lists and bounds.
struct Binned {
    TileGeom g;
    const wasabi_point *sorted;
    int64_t *tile_off;
    int32_t *tile_pts;
    double *cell_bound;
    bool ordered;
};

int bin_window(const wasabi_lut *lut, const wasabi_point *pts, int64_t n, int64_t ox, int64_t oy,
               int32_t nx, int32_t ny, Scratch &sc, hipStream_t s, Binned &b)
{
    b.g = make_geom(ox, oy, nx, ny);
    choose_lists(b.g);
    b.ordered = false;
    return bin_points(lut, pts, n, b.g, sc, s, &b.sorted, &b.tile_off, &b.tile_pts, &b.cell_bound, &b.ordered);
}

// Superposition of the window (ox, oy, nx, ny) from the lists of `b`, whose window holds this one
// with this one's origin on its tile grid.
int launch_window(const wasabi_lut *lut, const Binned &b, int64_t ox, int64_t oy, int32_t nx, int32_t ny,
                  void *out, int64_t ld, int mode, hipStream_t s, bool allow_pace, Scratch &sc,
                  int accumulate = 0)
{
    TileGeom g = make_geom(ox, oy, nx, ny);
    g.cell = b.g.cell;
    g.nlx = b.g.nlx;
    g.nly = b.g.nly;
    g.ltx0 = (int32_t)((ox - b.g.ox) / kT);
    g.lty0 = (int32_t)((oy - b.g.oy) / kT);
    TileArgs a = make_args(lut, b.sorted, b.tile_off, b.tile_pts, g, (float2 *)out, ld);
    a.cell_bound = b.cell_bound;
    a.stream_psi = mode == MODE_PSI && streams_past_cache(nx, ny);
    a.accumulate = mode == MODE_PSI && accumulate;
    // Plane pacing (bounded waits; see the dense kernel) when the lists are in plane order and
    // every tile of the grid is resident at once.  CGH_PACE=0 switches it off, CGH_PACE_SLACK sets
    // how many planes a tile may run ahead of the slowest one.
    static const int pace_env = getenv("CGH_PACE") ? atoi(getenv("CGH_PACE")) : 1;
    static const int slack_env = getenv("CGH_PACE_SLACK") ? atoi(getenv("CGH_PACE_SLACK")) : 5;
    int rc;
    if (allow_pace && pace_env && lut->dense && b.ordered && lut->L >= 3 && lut->n_tables <= kPaceMaxPlanes &&
        resident_capacity(lut->L, lut->prm.value_dtype, mode) >= (int64_t)g.ntx * g.nty) {
        int *done;
        const size_t bytes = sizeof(int) * (size_t)lut->n_tables * kPaceCounters;
        if ((rc = sc.alloc((void **)&done, bytes))) return rc;
        if ((rc = zero_words(done, (int64_t)lut->n_tables * kPaceCounters, s))) return rc;
        a.plane_done = done;
        a.pace_slack = std::max(1, slack_env);
    }
    if (mode == MODE_PSI) return launch_tile<MODE_PSI>(lut->L, lut->prm.value_dtype, a, s);
    return launch_tile<MODE_FUSED>(lut->L, lut->prm.value_dtype, a, s);
}

int superpose_impl(const wasabi_lut *lut, const wasabi_point *pts, int64_t n, int64_t ox,
                   int64_t oy, int32_t nx, int32_t ny, void *out, int64_t ld, int mode,
                   hipStream_t s, bool allow_pace = true, Scratch *ext = nullptr, int accumulate = 0)
{
    int rc = ext ? CGH_OK : prepare_pool();
    if (rc) return rc;
    Scratch local(s);
    Scratch &sc = ext ? *ext : local;
    Binned b;
    if ((rc = bin_window(lut, pts, n, ox, oy, nx, ny, sc, s, b))) return rc;
    return launch_window(lut, b, ox, oy, nx, ny, out, ld, mode, s, allow_pace, sc, accumulate);
}

int check_common(const wasabi_lut *lut, const wasabi_point *pts, int64_t n, int64_t ox, int64_t oy,
                 int32_t nx, int32_t ny, const void *out)
{
    if (!lut) return fail(CGH_EINVAL, "lut is NULL");
    if (n < 0 || n > INT32_MAX) return fail(CGH_EINVAL, "n out of range");
    if (n > 0 && !pts) return fail(CGH_EINVAL, "pts is NULL");
    if (!out) return fail(CGH_EINVAL, "output is NULL");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != lut->device) return fail(CGH_EINVAL, "LUT lives on device %d, current is %d", lut->device, dev);
    return check_window(lut->L, ox, oy, nx, ny);
}

int idwt_impl(const void *psi, int32_t nx, int32_t ny, int32_t levels, void *u, int64_t ld,
              hipStream_t s)
{
    const TileGeom g = make_geom(0, 0, nx, ny);
    TileArgs a = make_args(nullptr, nullptr, nullptr, nullptr, g, (float2 *)u, ld);
    a.in = (const float2 *)psi;
    const int64_t ntiles = (int64_t)g.ntx * g.nty;
    if (ntiles > INT32_MAX) return fail(CGH_EINVAL, "too many tiles");
    const dim3 grid((unsigned)ntiles);
    ProfScope prof("idwt", s);
    switch (levels) {
    case 1: hipLaunchKernelGGL(idwt_kernel<1>, grid, dim3(kThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL(idwt_kernel<2>, grid, dim3(kThreads), 0, s, a); break;
    case 3: hipLaunchKernelGGL(idwt_kernel<3>, grid, dim3(kThreads), 0, s, a); break;
    case 4: hipLaunchKernelGGL(idwt_kernel<4>, grid, dim3(kThreads), 0, s, a); break;
    case 5: hipLaunchKernelGGL(idwt_kernel<5>, grid, dim3(kThreads), 0, s, a); break;
    default: hipLaunchKernelGGL(idwt_kernel<6>, grid, dim3(kThreads), 0, s, a); break;
    }
    CGH_CHECK_LAUNCH("idwt_kernel");
    return CGH_OK;
}

}  // namespace

int64_t fused_scratch_bound(const wasabi_lut *lut, int64_t n, int32_t nx, int32_t ny, bool pacing)
{
    TileGeom g = make_geom(0, 0, nx, ny);
    choose_lists(g);
    const int64_t ntiles = (int64_t)g.nlx * g.nly;  // lists
    const int64_t nbins = (int64_t)lut->n_tables * sort_bands(lut, g) + 1;
    const int64_t bound = pair_bound(lut, n, g);
    auto r = scratch_round;
    // counts, offsets, lists, sorted points, the plane sort, the cell bounds (bin_points' order)
    int64_t t = r(4 * ntiles) + r(8 * (ntiles + 1)) + r(4 * bound) + r(16 * std::max<int64_t>(n, 1)) +
                radix_scratch(n, key_bits(nbins), 16) + r(8 * ntiles);
    if (use_matrix_path(n, ntiles)) {
        const int64_t cells = (n + chunk_pts(n) - 1) / chunk_pts(n) * ntiles;
        t += r(4 * cells) + r(8 * (cells + 1)) + scan_scratch(cells);
    } else {
        t += scan_scratch(ntiles);
        if (lut->dense)
            t += r(4 * n) + r(8 * (n + 1)) + scan_scratch(n) + r(8 * bound) + radix_scratch(bound, key_bits(ntiles), 8);
        else
            t += r(8 * ntiles);
    }
    if (pacing) t += r(4 * (int64_t)lut->n_tables * kPaceCounters);
    return t;
}

int hologram_fused_shared(const wasabi_lut *lut, const wasabi_point *pts, int64_t n, int32_t nx,
                          int32_t ny, void *u, hipStream_t s, void *arena, size_t arena_bytes)
{
    int rc = check_common(lut, pts, n, 0, 0, nx, ny, u);
    if (rc) return rc;
    if (lut->prm.wavelet != CGH_HAAR) return fail(CGH_EINVAL, "the fused path needs a Haar LUT");
    Scratch sc(s, arena, arena_bytes);
    return superpose_impl(lut, pts, n, 0, 0, nx, ny, u, nx, MODE_FUSED, s, false, &sc);
}

}  // namespace cgh

extern "C" int wasabi_superpose(const wasabi_lut *lut, const wasabi_point *pts, int64_t n,
                                int64_t ox, int64_t oy, int32_t nx, int32_t ny, void *psi,
                                int32_t accumulate, void *stream)
{
    using namespace cgh;
    int rc = check_common(lut, pts, n, ox, oy, nx, ny, psi);
    if (rc) return rc;
    if (accumulate != 0 && accumulate != 1) return fail(CGH_EINVAL, "accumulate must be 0 or 1");
    return superpose_impl(lut, pts, n, ox, oy, nx, ny, psi, nx, MODE_PSI, (hipStream_t)stream, true,
                          nullptr, accumulate);
}

extern "C" int wasabi_idwt(const void *psi, int32_t nx, int32_t ny, int32_t levels, void *u,
                           int64_t ld_u, void *stream)
{
    using namespace cgh;
    if (!psi || !u) return fail(CGH_EINVAL, "NULL pointer");
    if (levels < 1 || levels > 6) return fail(CGH_EINVAL, "levels must be 1..6");
    int rc = check_window(levels, 0, 0, nx, ny);
    if (rc) return rc;
    if (ld_u < nx) return fail(CGH_EINVAL, "ld_u < nx");
    const uintptr_t pb = (uintptr_t)psi, ub = (uintptr_t)u;
    const uintptr_t pe = pb + sizeof(float2) * (uintptr_t)nx * (uintptr_t)ny;
    const uintptr_t ue = ub + sizeof(float2) * ((uintptr_t)(ny - 1) * (uintptr_t)ld_u + (uintptr_t)nx);
    const bool in_place = psi == u && ld_u == nx;
    if (pb < ue && ub < pe && !in_place)
        return fail(CGH_EINVAL, "u overlaps psi without being the same contiguous array (in place needs u == psi, ld_u == nx)");
    hipStream_t s = (hipStream_t)stream;
    if (!in_place) return idwt_impl(psi, nx, ny, levels, u, ld_u, s);
    // In place.  A tile's pixels land where the Mallat layout keeps coefficients of other tiles
    // (the inverse is a global permutation of the field), so the field is first copied to scratch
    // and the inverse reads the copy: 8 nx ny bytes of scratch and twice the traffic of the
    // out-of-place call.
    if ((rc = prepare_pool())) return rc;
    Scratch sc(s);
    void *copy;
    if ((rc = sc.alloc(&copy, sizeof(float2) * (size_t)nx * ny))) return rc;
    CGH_TRY_HIP(hipMemcpyAsync(copy, psi, sizeof(float2) * (size_t)nx * ny, hipMemcpyDeviceToDevice, s));
    return idwt_impl(copy, nx, ny, levels, u, ld_u, s);
}

extern "C" int wasabi_hologram(const wasabi_lut *lut, const wasabi_point *pts, int64_t n,
                               int64_t ox, int64_t oy, int32_t nx, int32_t ny, int32_t sub,
                               void *u, int64_t ld_u, void *stream)
{
    using namespace cgh;
    int rc = check_common(lut, pts, n, ox, oy, nx, ny, u);
    if (rc) return rc;
    if (ld_u < nx) return fail(CGH_EINVAL, "ld_u < nx");
    const int B = lut->B;
    if (sub < 0 || sub % B) return fail(CGH_EINVAL, "sub must be 0 or a positive multiple of 2^L");
    hipStream_t s = (hipStream_t)stream;
    if (lut->prm.wavelet != CGH_HAAR) return coiflet_hologram(lut, pts, n, ox, oy, nx, ny, sub, u, ld_u, s);
    if (sub == 0) sub = std::max(nx, ny);
    if ((rc = prepare_pool())) return rc;
    const int32_t sx = std::min(sub, nx), sy = std::min(sub, ny);
    Scratch sc(s);
    float2 *psi;
    if ((rc = sc.alloc((void **)&psi, sizeof(float2) * (size_t)sx * sy))) return rc;
    // The points are binned once for the whole window when every sub-hologram starts on its tile
    // grid; otherwise per sub-hologram.
    const bool once = (sub % kT == 0) || (sx == nx && sy == ny);
    Binned b;
    if (once && (rc = bin_window(lut, pts, n, ox, oy, nx, ny, sc, s, b))) return rc;
    // Sec. 2, large-scale procedure: for every sub-hologram (s, t), shift the points
    // (x'_j = x_j - s N_h), superpose in the wavelet domain, invert into the hologram.
    for (int64_t t0 = 0; t0 < ny; t0 += sub) {
        for (int64_t s0 = 0; s0 < nx; s0 += sub) {
            const int32_t wx = (int32_t)std::min<int64_t>(sub, nx - s0);
            const int32_t wy = (int32_t)std::min<int64_t>(sub, ny - t0);
            if (once)
                rc = launch_window(lut, b, ox + s0, oy + t0, wx, wy, psi, wx, MODE_PSI, s, true, sc);
            else
                rc = superpose_impl(lut, pts, n, ox + s0, oy + t0, wx, wy, psi, wx, MODE_PSI, s);
            if (rc) return rc;
            float2 *uw = (float2 *)u + t0 * ld_u + s0;
            rc = idwt_impl(psi, wx, wy, lut->L, uw, ld_u, s);
            if (rc) return rc;
        }
    }
    return CGH_OK;
}

extern "C" int wasabi_hologram_fused(const wasabi_lut *lut, const wasabi_point *pts, int64_t n,
                                     int64_t ox, int64_t oy, int32_t nx, int32_t ny, void *u,
                                     int64_t ld_u, void *stream)
{
    using namespace cgh;
    int rc = check_common(lut, pts, n, ox, oy, nx, ny, u);
    if (rc) return rc;
    if (ld_u < nx) return fail(CGH_EINVAL, "ld_u < nx");
    if (lut->prm.wavelet != CGH_HAAR)
        return fail(CGH_EINVAL, "the fused path inverts Haar blocks on chip; a coiflet LUT needs wasabi_hologram");
    return superpose_impl(lut, pts, n, ox, oy, nx, ny, u, ld_u, MODE_FUSED, (hipStream_t)stream);
}


// ---- the fused hologram without allocation ---------------------------------------------------
// Scratch of wasabi_hologram_fused_noalloc: a file-scope device array, one copy on every device
// the library runs on, held until the process ends.  Host code never uses the array's name as a
// device address (on the host it only names the symbol): the address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace cgh {
namespace {

constexpr int kMaxDevices = 64;

int static_scratch(void **out)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = -1;
    CGH_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CGH_EINVAL, "device %d beyond the %d the library tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return fail(CGH_EHIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
        }
        addr[dev] = p;
    }
    *out = addr[dev];
    return CGH_OK;
}

}  // namespace
}  // namespace cgh

extern "C" int wasabi_hologram_fused_noalloc(const wasabi_lut *lut, const wasabi_point *pts, int64_t n,
                                             int64_t ox, int64_t oy, int32_t nx, int32_t ny, void *u,
                                             int64_t ld_u, void *stream)
{
    using namespace cgh;
    int rc = check_common(lut, pts, n, ox, oy, nx, ny, u);
    if (rc) return rc;
    if (ld_u < nx) return fail(CGH_EINVAL, "ld_u < nx");
    if (lut->prm.wavelet != CGH_HAAR)
        return fail(CGH_EINVAL, "the fused path inverts Haar blocks on chip; a coiflet LUT needs wasabi_hologram");
    const int64_t need = fused_scratch_bound(lut, n, nx, ny, true);
    if (need > (int64_t)kStaticScratchBytes)
        return fail(CGH_ENOMEM, "%lld points on a %d x %d window need %lld bytes of scratch; the static buffer holds %zu",
                    (long long)n, nx, ny, (long long)need, kStaticScratchBytes);
    void *buf = nullptr;
    if ((rc = static_scratch(&buf))) return rc;
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s, buf, kStaticScratchBytes);
    return superpose_impl(lut, pts, n, ox, oy, nx, ny, u, ld_u, MODE_FUSED, s, true, &sc);
}
