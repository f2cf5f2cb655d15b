// Internal definitions shared by the translation units of libcgh.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "cgh.h"

namespace cgh {

// ---------------------------------------------------------------------------------------------
// Error reporting: every public entry point returns a cgh_status and leaves a thread-local text.
// ---------------------------------------------------------------------------------------------
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define CGH_TRY_HIP(call)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::cgh::fail(CGH_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));       \
    } while (0)

#define CGH_CHECK_LAUNCH(name)                                                                 \
    do {                                                                                       \
        hipError_t e_ = hipGetLastError();                                                     \
        if (e_ != hipSuccess)                                                                  \
            return ::cgh::fail(CGH_EHIP, "launch of %s failed: %s", name, hipGetErrorString(e_)); \
    } while (0)

// Stream-ordered scratch: allocated from the device's default pool on `stream` and returned to
// it on the same stream when the guard goes out of scope.
// With an arena, allocations are carved (256-byte aligned) from that caller-owned device buffer
// instead, and nothing is freed: work on `stream` orders the reuse of the arena.  Without one, the
// first allocation fails with CGH_EINVAL while `stream` is being captured into a HIP graph.
class Scratch {
  public:
    explicit Scratch(hipStream_t s) : stream_(s) {}
    Scratch(hipStream_t s, void *arena, size_t cap) : stream_(s), arena_((char *)arena), cap_(cap) {}
    ~Scratch();
    // Returns CGH_OK or CGH_ENOMEM/CGH_EHIP; *p receives device memory of `bytes` bytes.
    int alloc(void **p, size_t bytes);

  private:
    hipStream_t stream_;
    std::vector<void *> ptrs_;
    char *arena_ = nullptr;
    size_t cap_ = 0, used_ = 0;
    bool capture_checked_ = false;
};

// Keeps the default pool's memory cached between calls (release threshold = unlimited) and stops it
// from making one stream wait for another to reuse memory.
int prepare_pool();

// Exclusive scan of `count` int32 values into int64 offsets (count + 1 values) on stream s.
int scan_counts(const int32_t *counts, int64_t count, int64_t *off, Scratch &sc, hipStream_t s);

// Records a HIP event pair around the enclosed launches on `s` while tracing is enabled.
class ProfScope {
  public:
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();

  private:
    const char *name_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr;
};

// ---------------------------------------------------------------------------------------------
// Coefficient LUT, device layout.
//
// Plane d's W x W table is cut into nb x nb Haar blocks of B x B pixels (B = 2^L).  Because the
// Haar transform of an aligned B x B block involves only that block, each block's coefficients
// are stored with the block: in-block position "code" = ir * B + ic of the block's own L-level
// Mallat layout.  The kept entries of a plane are ordered by (block row, block column, code) and
// carry a 16-bit key = block_column * BS(L) + code, where BS(L) is the (padded) block stride of
// the on-chip tile buffer used by the superposition kernels.  For an entry of block row br,
// the tile-buffer address is therefore  row_base(br) + key  with one uniform row_base per row.
// blk_off[d] holds nb*nb + 1 offsets: entries of block (br, bc) are [blk_off[br*nb+bc],
// blk_off[br*nb+bc+1]) relative to the plane's first entry.
// ---------------------------------------------------------------------------------------------
// Selectivity from which a LUT also gets the dense layout (and the superposition uses it): at
// gamma ~ 0.35 and above most codes of an occupied block are kept, so whole blocks cost about as
// many bytes as (value, key) entries and need no keys, no LDS atomics and no fixed point.
constexpr double kDenseGamma = 0.35;

// On-chip tile buffer layout: block (r, c) of a tile starts at r * row_stride + c * block_stride.
// The pads decide how the LDS banks of equal in-block codes of neighbouring blocks and block rows
// line up; these values minimise the bank conflicts of the superposition's scattered atomic adds
// (a model of the 64-lane adds over the kept entries of real tables, for 32 and 64 banks).  L = 4
// has none: its unpadded 64 x 64 tile of 8-byte words is exactly 32 KiB, so five tiles share a
// compute unit's 160 KiB instead of four, which measured faster than the pads' fewer conflicts.
__host__ __device__ constexpr int block_stride(int L)
{
    return L <= 2 ? (1 << (2 * L)) + (1 << L) : (L == 4 ? 256 : (1 << (2 * L)) + (1 << (L - 2)));
}

__host__ __device__ constexpr int row_pad(int L)
{
    return L == 3 ? 32 : 0;
}

struct DepthDesc {
    int32_t W;            // table side
    int32_t nb;           // W / B
    int32_t br0, br1;     // block rows holding kept entries: [br0, br1)
    int32_t bc0, bc1;     // block columns holding kept entries: [bc0, bc1)
    float cmax;           // largest |re| or |im| of the plane's stored values
    int32_t pad;
    int64_t entry_base;   // first entry of the plane in values/keys
    int64_t blkoff_base;  // first element of the plane's blk_off array
    int64_t dense_base;   // dense layout: first coefficient of the plane in dense values
    int64_t rows_base;    // dense layout: first DenseRow of the plane (nb rows)
};

// Dense layout (kept when gamma is large): every Haar block of a block row between the first and
// the last block holding kept entries is stored whole (B*B coefficients, zeros where dropped),
// block after block, so the blocks a tile needs from one table block row are one contiguous run.
// Zero values stored after the dense tables: the superposition reads them in place of table blocks
// that a pair does not cover, so every pair issues the same loads.
constexpr int kDenseZero = 512;

struct DenseRow {
    int32_t lo, hi;  // stored blocks [lo, hi) of this block row
    int32_t off;     // first coefficient of block lo, relative to the plane's dense_base
    int32_t pad;
};

}  // namespace cgh

// Tables: one per plane, or with phase tables 4^L per plane (table t = d 4^L + sy 2^L + sx holds
// plane d's PSF centred sx columns right of and sy rows below the table centre).  Every per-table
// vector below has n_tables entries.
struct wasabi_lut {
    wasabi_lut_params prm;
    int device;
    int L, B;
    int P;                            // tables per plane: 1, or 4^L with phase tables
    int n_tables;                     // n_depth * P
    std::vector<double> z, R;
    std::vector<int32_t> W;
    std::vector<int64_t> Nr;
    std::vector<int64_t> entry_off;   // n_tables + 1
    std::vector<cgh::DepthDesc> desc_host;
    int64_t total_entries;
    int32_t max_span_px;              // largest occupied extent of any plane, pixels
    cgh::DepthDesc *desc;             // device, n_tables
    int32_t *blk_off;                 // device
    void *values;                     // device: float2 (F32) or uint32 packed pair (F16, BF16)
    uint16_t *keys;                   // device
    int32_t *wkeys;                   // device, sparse layout only: each entry's byte offset in the
                                      // superposition's on-chip tile buffer, (table block row * row
                                      // stride + key) * 8, for a table whose block (0, 0) sits on
                                      // tile block (0, 0)
    bool dense;                       // dense layout present (used by the superposition)
    void *dense_values;               // device, same element type as values
    int64_t dense_zero;               // first of kDenseZero zero values after the dense tables
    cgh::DenseRow *dense_rows;        // device
    size_t device_bytes;
};

namespace cgh {
// Geometry of the planes (Sec. 2, step 1); fills z, R, W, Nr of `lut`.  Returns CGH_OK or CGH_EINVAL.
int lut_geometry(wasabi_lut *lut);
int validate_params(const wasabi_lut_params *prm);

// Analysis filter bank of `wavelet` (CGH_HAAR or CGH_COIF1) into lo/hi (8 entries each); returns taps.
int wavelet_filters(int wavelet, double *lo, double *hi);

// wasabi_hologram for a coiflet LUT: every sub-hologram grown by a halo, superposed, inverted with
// the periodised synthesis filter bank, its centre copied to u (coiflet.hip).
int coiflet_hologram(const wasabi_lut *lut, const wasabi_point *pts, int64_t n, int64_t ox, int64_t oy,
                     int32_t nx, int32_t ny, int32_t sub, void *u, int64_t ld_u, hipStream_t s);

// Upper bound (bytes) of the device scratch wasabi_hologram_fused takes for n points on an nx x ny
// window (any origin), with or without the plane-pacing counters.
int64_t fused_scratch_bound(const wasabi_lut *lut, int64_t n, int32_t nx, int32_t ny, bool pacing);

// wasabi_hologram_fused at origin (0, 0), u contiguous, without plane pacing (for work that shares
// the device with other streams, where the tiles of one launch cannot count on being co-resident),
// its scratch carved from `arena` (at least fused_scratch_bound bytes).
int hologram_fused_shared(const wasabi_lut *lut, const wasabi_point *pts, int64_t n, int32_t nx,
                          int32_t ny, void *u, hipStream_t s, void *arena, size_t arena_bytes);
}  // namespace cgh
