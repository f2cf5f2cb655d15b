// Eq.(1): u(x_h, y_h) = sum_j a_j exp(i 2 pi r_hj / lambda), the direct superposition of point
// sources, as a VALU kernel for gfx950.
//
// Work split, FULL window: a 256-thread workgroup owns a 64 x 16 pixel tile; thread t owns column
// t % 64 and rows t / 64 + 4k (k = 0..3), so the x-distance is shared by its four pixels.  Points
// stream through LDS in chunks of 256.
// CIRC window: points are first binned by 64 x 64 tile (the bounding box of their disk), and a
// workgroup sums only its tile's list (16 pixels per thread), so the cost follows the number of
// (pixel, point) pairs inside the disks rather than pixels x points.
//
// Precision: the phase r / lambda reaches thousands of revolutions, so it is formed in FP64 and
// reduced to its fractional part before the sine and cosine.  For complex64 output r comes from
// an FP32 reciprocal square root refined by one FP64 Newton step (relative error ~1e-14), the
// reduced phase goes to the hardware sine/cosine (argument in revolutions) and sums are FP32.
// For complex128 output everything is FP64.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "common.hpp"

namespace cgh {
namespace {

constexpr int kTX = 64, kTY = 16, kRows = 4, kThreads = 256;

// sin(2 pi f) and cos(2 pi f) in FP64 for a phase already reduced to f in [0, 1).  Quarter-period
// reduction: 2 pi f = (pi / 2)(q + r) with q = rint(4 f) and |r| <= 1/2 (exact in FP64), then the
// Taylor series of sin and cos about 0 on |x| = |pi r / 2| <= pi / 4 in Horner form in x^2, up to
// x^17 and x^16 (the first omitted terms are below 1e-17), and the quadrant q mod 4 swaps and
// negates them.  Error against a 120-bit reference: below 1.6e-16 absolute on f in [0, 1).  A
// general-argument sincospi spends more instructions on reduction that this phase does not need.
__device__ inline void sincos_2pi(double f, double *sn, double *cs)
{
    const double u = 4.0 * f;
    const double q = rint(u);
    const double x = (u - q) * 1.5707963267948966;  // (pi / 2) r
    const double x2 = x * x;
    double ps = 2.8114572543455206e-15;             // 1/17!
    ps = fma(ps, x2, -7.647163731819816e-13);       // -1/15!
    ps = fma(ps, x2, 1.6059043836821613e-10);       // 1/13!
    ps = fma(ps, x2, -2.505210838544172e-08);       // -1/11!
    ps = fma(ps, x2, 2.7557319223985893e-06);       // 1/9!
    ps = fma(ps, x2, -0.0001984126984126984);       // -1/7!
    ps = fma(ps, x2, 0.008333333333333333);         // 1/5!
    ps = fma(ps, x2, -0.16666666666666666);         // -1/3!
    const double s = fma(ps * x2, x, x);            // x + x^3 (...)
    double pc = 4.779477332387385e-14;              // 1/16!
    pc = fma(pc, x2, -1.1470745597729725e-11);      // -1/14!
    pc = fma(pc, x2, 2.08767569878681e-09);         // 1/12!
    pc = fma(pc, x2, -2.755731922398589e-07);       // -1/10!
    pc = fma(pc, x2, 2.48015873015873e-05);         // 1/8!
    pc = fma(pc, x2, -0.001388888888888889);        // -1/6!
    pc = fma(pc, x2, 0.041666666666666664);         // 1/4!
    pc = fma(pc, x2, -0.5);                         // -1/2!
    const double c = fma(pc, x2, 1.0);
    const int quadrant = (int)q & 3;
    const double a = (quadrant & 1) ? c : s, b = (quadrant & 1) ? s : c;
    *sn = (quadrant & 2) ? -a : a;                  // 0: s  1: c  2: -s  3: -c
    *cs = (quadrant == 1 || quadrant == 2) ? -b : b;  // 0: c  1: -s  2: -c  3: s
}

struct DirectArgs {
    const double4 *pts;
    int64_t n;
    int32_t nx, ny;
    int64_t ox, oy;
    double pitch, inv_lambda, tan2;  // tan2 = tan(theta)^2
    void *out;
    int64_t ld;
    int64_t chunk;        // points per blockIdx.z slice (n when the points are not split)
    int64_t part_stride;  // split: slice z writes its partial field at out + z * part_stride (ld = nx)
};

// A workgroup sums a 64 x 4 ROWS pixel tile: wave w owns rows w, w + 4, ... of it, lane l column l.
// ROWS = 4 amortises each point's LDS read and x distance over four pixels; ROWS = 1 gives four
// times as many workgroups for holograms too small to fill the chip otherwise.
template <bool CIRC, bool F64, int ROWS>
__global__ __launch_bounds__(kThreads) void direct_kernel(DirectArgs a)
{
    constexpr int TY = 4 * ROWS;
    __shared__ double4 sp[kThreads];      // x, y, z^2, amplitude
    __shared__ double sr2[kThreads];      // disk radius^2 (metres^2)
    __shared__ int swave[kThreads / 64];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int col = blockIdx.x * kTX + lane;
    const int row0 = blockIdx.y * TY + wave;
    const double xh = (double)(a.ox + col) * a.pitch;
    double yh[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; k++) yh[k] = (double)(a.oy + row0 + 4 * k) * a.pitch;

    // tile rectangle in metres (pixel centres), for culling
    const double tx0 = (double)(a.ox + (int64_t)blockIdx.x * kTX) * a.pitch;
    const double tx1 = tx0 + (kTX - 1) * a.pitch;
    const double ty0 = (double)(a.oy + (int64_t)blockIdx.y * TY) * a.pitch;
    const double ty1 = ty0 + (TY - 1) * a.pitch;

    double accd_re[ROWS], accd_im[ROWS];
    float accf_re[ROWS], accf_im[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; k++) {
        accd_re[k] = accd_im[k] = 0.0;
        accf_re[k] = accf_im[k] = 0.0f;
    }

    // this workgroup's slice of the points (all of them unless the sum is split over blockIdx.z)
    const int64_t j0 = (int64_t)blockIdx.z * a.chunk, j1 = min(a.n, j0 + a.chunk);
    for (int64_t base = j0; base < j1; base += kThreads) {
        const int64_t j = base + tid;
        bool keep = false;
        double4 p = make_double4(0, 0, 0, 0);
        double r2 = 0.0;
        if (j < j1) {
            p = a.pts[j];
            r2 = p.z * p.z * a.tan2;
            keep = true;
            if (CIRC) {
                // distance from the disk centre to the tile rectangle; the small margin keeps
                // every point whose exact per-pixel test could pass
                const double cx = fmin(fmax(p.x, tx0), tx1), cy = fmin(fmax(p.y, ty0), ty1);
                const double ddx = p.x - cx, ddy = p.y - cy;
                keep = ddx * ddx + ddy * ddy < r2 * (1.0 + 1e-9);
            }
        }
        // order-preserving compaction of the kept points of this chunk
        const uint64_t m = __ballot(keep);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) swave[wave] = __popcll(m);
        __syncthreads();
        int off = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; w++) {
            off += (w < wave) ? swave[w] : 0;
            total += swave[w];
        }
        if (keep) {
            const int s = off + before;
            sp[s] = make_double4(p.x, p.y, p.z * p.z, p.w);
            sr2[s] = r2;
        }
        __syncthreads();

        for (int k = 0; k < total; k++) {
            const double4 q = sp[k];
            const double dx = xh - q.x;
            const double dx2 = dx * dx;
#pragma unroll
            for (int rr = 0; rr < ROWS; rr++) {
                const double dy = yh[rr] - q.y;
                const double rho2 = fma(dy, dy, dx2);
                const double d2 = rho2 + q.z;
                if (F64) {
                    double amp = q.w;
                    if (CIRC && !(rho2 < sr2[k])) amp = 0.0;
                    const double t = sqrt(d2) * a.inv_lambda;
                    const double f = t - floor(t);
                    double s, c;
                    sincos_2pi(f, &s, &c);
                    accd_re[rr] = fma(amp, c, accd_re[rr]);
                    accd_im[rr] = fma(amp, s, accd_im[rr]);
                } else {
                    float amp = (float)q.w;
                    if (CIRC && !(rho2 < sr2[k])) amp = 0.0f;
                    const float y = __builtin_amdgcn_rsqf((float)d2);
                    const double r0 = d2 * (double)y;
                    const double res = fma(-r0, r0, d2);
                    const double r = fma(res, 0.5 * (double)y, r0);
                    const double t = r * a.inv_lambda;
                    const float f = (float)(t - floor(t));
                    const float s = __builtin_amdgcn_sinf(f);  // sin(2 pi f)
                    const float c = __builtin_amdgcn_cosf(f);
                    accf_re[rr] = fmaf(amp, c, accf_re[rr]);
                    accf_im[rr] = fmaf(amp, s, accf_im[rr]);
                }
            }
        }
        __syncthreads();
    }

    if (col < a.nx) {
#pragma unroll
        for (int rr = 0; rr < ROWS; rr++) {
            const int row = row0 + 4 * rr;
            if (row >= a.ny) continue;
            const int64_t at = (int64_t)blockIdx.z * a.part_stride + (int64_t)row * a.ld + col;
            if (F64) {
                ((double2 *)a.out)[at] = make_double2(accd_re[rr], accd_im[rr]);
            } else {
                ((float2 *)a.out)[at] = make_float2(accf_re[rr], accf_im[rr]);
            }
        }
    }
}

// Sums the nsplit partial fields (nx x ny each, contiguous) in slice order into the output.
template <typename T>
__global__ __launch_bounds__(256) void sum_parts_kernel(const T *part, int nsplit, int32_t nx, int32_t ny,
                                                        T *out, int64_t ld)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)nx * ny) return;
    const int64_t plane = (int64_t)nx * ny;
    T acc = part[i];
    for (int z = 1; z < nsplit; ++z) {
        const T v = part[z * plane + i];
        acc.x += v.x;
        acc.y += v.y;
    }
    out[(i / nx) * ld + i % nx] = acc;
}

// ---- circ() window at scale: points binned by 64 x 16 tile (tiles their disk reaches), then each
//      tile sums only its own points with the same thread layout as above. ----

struct BinArgs {
    const double4 *pts;
    int64_t n;
    int32_t nx, ny, ntx, nty;
    int64_t ox, oy;
    double pitch, tan_t;
};

// Tile range of the disk's bounding box (pixels, one pixel of margin); false if it misses the window.
__device__ inline bool disk_tiles(const double4 &p, const BinArgs &b, double &cx, double &cy, double &R,
                                  int &ty0, int &ty1, int &tx0, int &tx1)
{
    if (!(p.z > 0.0) || !isfinite(p.x) || !isfinite(p.y)) return false;
    R = p.z * b.tan_t / b.pitch;
    cx = p.x / b.pitch - (double)b.ox;
    cy = p.y / b.pitch - (double)b.oy;
    const double x0 = ceil(cx - R - 1.0), x1 = floor(cx + R + 1.0);
    const double y0 = ceil(cy - R - 1.0), y1 = floor(cy + R + 1.0);
    if (x1 < 0 || y1 < 0 || x0 > b.nx - 1 || y0 > b.ny - 1) return false;
    tx0 = (int)(fmax(x0, 0.0) / kTX);
    tx1 = (int)(fmin(x1, (double)(b.nx - 1)) / kTX) + 1;
    ty0 = (int)(fmax(y0, 0.0) / kTY);
    ty1 = (int)(fmin(y1, (double)(b.ny - 1)) / kTY) + 1;
    return true;
}

// Does the disk reach tile (ty, tx)?  Distance from the centre to the tile's rectangle of pixel
// centres, with a one-pixel margin (the exact per-pixel test runs in the summation kernel).
__device__ inline bool disk_hits(double cx, double cy, double R, int ty, int tx)
{
    const double rx0 = tx * kTX, rx1 = rx0 + kTX - 1, ry0 = ty * kTY, ry1 = ry0 + kTY - 1;
    const double dx = cx - fmin(fmax(cx, rx0), rx1), dy = cy - fmin(fmax(cy, ry0), ry1);
    return dx * dx + dy * dy < (R + 1.0) * (R + 1.0);
}

__global__ void disk_count_kernel(BinArgs b, int32_t *counts)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= b.n) return;
    double cx, cy, R;
    int ty0, ty1, tx0, tx1;
    if (!disk_tiles(b.pts[j], b, cx, cy, R, ty0, ty1, tx0, tx1)) return;
    for (int ty = ty0; ty < ty1; ++ty)
        for (int tx = tx0; tx < tx1; ++tx)
            if (disk_hits(cx, cy, R, ty, tx)) atomicAdd(&counts[(int64_t)ty * b.ntx + tx], 1);
}

__global__ void disk_fill_kernel(BinArgs b, unsigned long long *cursor, int32_t *list)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= b.n) return;
    double cx, cy, R;
    int ty0, ty1, tx0, tx1;
    if (!disk_tiles(b.pts[j], b, cx, cy, R, ty0, ty1, tx0, tx1)) return;
    for (int ty = ty0; ty < ty1; ++ty)
        for (int tx = tx0; tx < tx1; ++tx)
            if (disk_hits(cx, cy, R, ty, tx)) {
                const unsigned long long slot = atomicAdd(&cursor[(int64_t)ty * b.ntx + tx], 1ull);
                list[slot] = (int32_t)j;
            }
}

template <bool F64>
__global__ __launch_bounds__(256) void direct_binned_kernel(DirectArgs a, int32_t ntx,
                                                            const int64_t *tile_off,
                                                            const int32_t *list)
{
    constexpr int ROWS = kRows;
    __shared__ double4 sp[256];
    __shared__ double sr2[256];
    const int tile = blockIdx.x;
    const int ty = tile / ntx, tx = tile - ty * ntx;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = tx * kTX + lane;
    const int row0 = ty * kTY + wave;
    const double xh = (double)(a.ox + col) * a.pitch;
    double accd_re[ROWS], accd_im[ROWS];
    float accf_re[ROWS], accf_im[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; k++) {
        accd_re[k] = accd_im[k] = 0.0;
        accf_re[k] = accf_im[k] = 0.0f;
    }
    const int64_t p0 = tile_off[tile], p1 = tile_off[tile + 1];
    for (int64_t base = p0; base < p1; base += 256) {
        const int cnt = (int)min((int64_t)256, p1 - base);
        if (tid < cnt) {
            const double4 p = a.pts[list[base + tid]];
            sp[tid] = make_double4(p.x, p.y, p.z * p.z, p.w);
            sr2[tid] = p.z * p.z * a.tan2;
        }
        __syncthreads();
        for (int k = 0; k < cnt; k++) {
            const double4 q = sp[k];
            const double r2lim = sr2[k];
            const double dx = xh - q.x;
            const double dx2 = dx * dx;
#pragma unroll
            for (int rr = 0; rr < ROWS; rr++) {
                const double yh = (double)(a.oy + row0 + 4 * rr) * a.pitch;
                const double dy = yh - q.y;
                const double rho2 = fma(dy, dy, dx2);
                const double d2 = rho2 + q.z;
                if (F64) {
                    const double amp = (rho2 < r2lim) ? q.w : 0.0;
                    const double t = sqrt(d2) * a.inv_lambda;
                    double s, c;
                    sincos_2pi(t - floor(t), &s, &c);
                    accd_re[rr] = fma(amp, c, accd_re[rr]);
                    accd_im[rr] = fma(amp, s, accd_im[rr]);
                } else {
                    const float amp = (rho2 < r2lim) ? (float)q.w : 0.0f;
                    const float y = __builtin_amdgcn_rsqf((float)d2);
                    const double r0 = d2 * (double)y;
                    const double res = fma(-r0, r0, d2);
                    const double r = fma(res, 0.5 * (double)y, r0);
                    const double t = r * a.inv_lambda;
                    const float f = (float)(t - floor(t));
                    accf_re[rr] = fmaf(amp, __builtin_amdgcn_cosf(f), accf_re[rr]);
                    accf_im[rr] = fmaf(amp, __builtin_amdgcn_sinf(f), accf_im[rr]);
                }
            }
        }
        __syncthreads();
    }
    if (col < a.nx) {
#pragma unroll
        for (int rr = 0; rr < ROWS; rr++) {
            const int row = row0 + 4 * rr;
            if (row >= a.ny) continue;
            if (F64) ((double2 *)a.out)[(int64_t)row * a.ld + col] = make_double2(accd_re[rr], accd_im[rr]);
            else ((float2 *)a.out)[(int64_t)row * a.ld + col] = make_float2(accf_re[rr], accf_im[rr]);
        }
    }
}

int direct_binned(const DirectArgs &a, double tan_t, bool f64, hipStream_t s)
{
    int rc = prepare_pool();
    if (rc) return rc;
    BinArgs b;
    b.pts = a.pts;
    b.n = a.n;
    b.nx = a.nx;
    b.ny = a.ny;
    b.ntx = (a.nx + kTX - 1) / kTX;
    b.nty = (a.ny + kTY - 1) / kTY;
    b.ox = a.ox;
    b.oy = a.oy;
    b.pitch = a.pitch;
    b.tan_t = tan_t;
    const int64_t ntiles = (int64_t)b.ntx * b.nty;
    if (ntiles > INT32_MAX) return fail(CGH_EINVAL, "too many tiles");
    Scratch sc(s);
    int32_t *counts, *list;
    int64_t *off;
    unsigned long long *cursor;
    if ((rc = sc.alloc((void **)&counts, sizeof(int32_t) * ntiles))) return rc;
    if ((rc = sc.alloc((void **)&off, sizeof(int64_t) * (ntiles + 1)))) return rc;
    if ((rc = sc.alloc((void **)&cursor, sizeof(unsigned long long) * ntiles))) return rc;
    CGH_TRY_HIP(hipMemsetAsync(counts, 0, sizeof(int32_t) * ntiles, s));
    const unsigned pblocks = (unsigned)((a.n + 255) / 256);
    if (a.n > 0) {
        hipLaunchKernelGGL(disk_count_kernel, dim3(pblocks), dim3(256), 0, s, b, counts);
        CGH_CHECK_LAUNCH("disk_count_kernel");
    }
    if ((rc = scan_counts(counts, ntiles, off, sc, s))) return rc;
    // the list length depends on the points' depths, which only the device holds: read the total
    // back (one 8-byte copy, one synchronisation) and size the list exactly
    int64_t total = 0;
    CGH_TRY_HIP(hipMemcpyAsync(&total, off + ntiles, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CGH_TRY_HIP(hipStreamSynchronize(s));
    if ((rc = sc.alloc((void **)&list, sizeof(int32_t) * std::max<int64_t>(total, 1)))) return rc;
    if (a.n > 0) {
        CGH_TRY_HIP(hipMemcpyAsync(cursor, off, sizeof(int64_t) * ntiles, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(disk_fill_kernel, dim3(pblocks), dim3(256), 0, s, b, cursor, list);
        CGH_CHECK_LAUNCH("disk_fill_kernel");
    }
    ProfScope prof("direct", s);
    if (f64) hipLaunchKernelGGL(direct_binned_kernel<true>, dim3((unsigned)ntiles), dim3(256), 0, s, a, b.ntx, off, list);
    else hipLaunchKernelGGL(direct_binned_kernel<false>, dim3((unsigned)ntiles), dim3(256), 0, s, a, b.ntx, off, list);
    CGH_CHECK_LAUNCH("direct_binned_kernel");
    return CGH_OK;
}

}  // namespace
}  // namespace cgh

extern "C" int cgh_direct(const double *pts, int64_t n, int32_t nx, int32_t ny, int64_t ox,
                          int64_t oy, double pitch, double wavelength, int32_t window,
                          int32_t out_dtype, void *out, int64_t ld_out, void *stream)
{
    using namespace cgh;
    if (n < 0 || nx < 1 || ny < 1 || ld_out < nx) return fail(CGH_EINVAL, "bad sizes");
    if (!(pitch > 0) || !(wavelength > 0) || !(wavelength < 2 * pitch))
        return fail(CGH_EINVAL, "need 0 < wavelength < 2 * pitch");
    if (window != CGH_FULL && window != CGH_CIRC) return fail(CGH_EINVAL, "unknown window");
    if (out_dtype != CGH_C64 && out_dtype != CGH_C128) return fail(CGH_EINVAL, "unknown out_dtype");
    if (!out || (n > 0 && !pts)) return fail(CGH_EINVAL, "NULL pointer");
    if ((int64_t)nx + ox > (INT64_C(1) << 40) || (int64_t)ny + oy > (INT64_C(1) << 40))
        return fail(CGH_EINVAL, "window origin out of range");
    hipStream_t s = (hipStream_t)stream;
    const double sin_t = wavelength / (2.0 * pitch);
    DirectArgs a;
    a.pts = (const double4 *)pts;
    a.n = n;
    a.nx = nx;
    a.ny = ny;
    a.ox = ox;
    a.oy = oy;
    a.pitch = pitch;
    a.inv_lambda = 1.0 / wavelength;
    a.tan2 = sin_t * sin_t / (1.0 - sin_t * sin_t);
    a.out = out;
    a.ld = ld_out;
    a.chunk = std::max<int64_t>(n, 1);
    a.part_stride = 0;
    const bool f64 = out_dtype == CGH_C128, circ = window == CGH_CIRC;
    dim3 grid((nx + kTX - 1) / kTX, (ny + kTY - 1) / kTY);
    // circ() with fewer than 8 workgroups per CU of 64 x 16 pixels: tiles of 64 x 4 instead, which
    // also cull the points more finely (512^2, N = 10^3: complex64 0.115 -> 0.090 ms, complex128
    // 0.347 -> 0.255 ms).  The full window gains nothing from it (complex128 0.60 -> 0.62 ms).
    const bool one_row = circ && (int64_t)grid.x * grid.y < 2048;
    const dim3 grid1((nx + kTX - 1) / kTX, (ny + 3) / 4);
    // circ(): cull every point against every tile while that is cheap, else bin first
    // (CGH_DIRECT_BIN=1 / 0 forces / forbids binning, for tests and measurements)
    const char *force = getenv("CGH_DIRECT_BIN");
    const bool bin = force ? atoi(force) != 0 : (double)n * grid.x * grid.y > 2e9;
    if (circ && bin) return direct_binned(a, sin_t / std::sqrt(1.0 - sin_t * sin_t), f64, s);
    if (grid.y > 65535) return fail(CGH_EINVAL, "ny too large");
    // The full window on fewer than 4 workgroups per CU: the points are split over up to 4 slices
    // (blockIdx.z), each summing into a partial field, and the partial fields are added in slice
    // order afterwards (512^2, N = 10^3: one wave per SIMD otherwise).
    int nsplit = 1;
    const int64_t wgs = (int64_t)grid.x * grid.y;
    if (!circ && wgs < 1024) nsplit = (int)std::min<int64_t>(std::min<int64_t>(4, (1024 + wgs - 1) / wgs), (n + 255) / 256);
    nsplit = std::max(nsplit, 1);
    ProfScope prof("direct", s);
    if (nsplit > 1) {
        int rc = prepare_pool();
        if (rc) return rc;
        Scratch sc(s);
        const size_t elem = f64 ? sizeof(double2) : sizeof(float2);
        void *part;
        if ((rc = sc.alloc(&part, elem * (size_t)nsplit * nx * ny))) return rc;
        a.out = part;
        a.ld = nx;
        a.part_stride = (int64_t)nx * ny;
        a.chunk = (n + nsplit - 1) / nsplit;
        const dim3 gz(grid.x, grid.y, (unsigned)nsplit);
        if (f64) hipLaunchKernelGGL((direct_kernel<false, true, kRows>), gz, dim3(kThreads), 0, s, a);
        else hipLaunchKernelGGL((direct_kernel<false, false, kRows>), gz, dim3(kThreads), 0, s, a);
        CGH_CHECK_LAUNCH("direct_kernel");
        const unsigned rb = (unsigned)(((int64_t)nx * ny + 255) / 256);
        if (f64)
            hipLaunchKernelGGL(sum_parts_kernel<double2>, dim3(rb), dim3(256), 0, s, (const double2 *)part, nsplit, nx, ny,
                               (double2 *)out, ld_out);
        else
            hipLaunchKernelGGL(sum_parts_kernel<float2>, dim3(rb), dim3(256), 0, s, (const float2 *)part, nsplit, nx, ny,
                               (float2 *)out, ld_out);
        CGH_CHECK_LAUNCH("sum_parts_kernel");
        return CGH_OK;
    }
    if (one_row && f64) {
        hipLaunchKernelGGL((direct_kernel<true, true, 1>), grid1, dim3(kThreads), 0, s, a);
    } else if (one_row) {
        hipLaunchKernelGGL((direct_kernel<true, false, 1>), grid1, dim3(kThreads), 0, s, a);
    } else if (circ && f64) {
        hipLaunchKernelGGL((direct_kernel<true, true, kRows>), grid, dim3(kThreads), 0, s, a);
    } else if (circ) {
        hipLaunchKernelGGL((direct_kernel<true, false, kRows>), grid, dim3(kThreads), 0, s, a);
    } else if (f64) {
        hipLaunchKernelGGL((direct_kernel<false, true, kRows>), grid, dim3(kThreads), 0, s, a);
    } else {
        hipLaunchKernelGGL((direct_kernel<false, false, kRows>), grid, dim3(kThreads), 0, s, a);
    }
    CGH_CHECK_LAUNCH("direct_kernel");
    return CGH_OK;
}
