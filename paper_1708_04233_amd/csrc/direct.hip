// Eq.(1): u(x_h, y_h) = sum_j a_j exp(i 2 pi r_hj / lambda), the direct superposition of point
// sources, as a VALU kernel for gfx950.
//
// Work split: a 256-thread workgroup owns a 64 x 16 pixel tile; thread t owns column t % 64 and
// rows t / 64 + 4k (k = 0..3), so the x-distance is shared by its four pixels.  Points stream
// through LDS in chunks of 256; with the circ() window each chunk is first culled against the
// tile (a point whose disk misses the whole tile is dropped before any per-pixel work) and the
// survivors are compacted in their original order, so sums are deterministic.
//
// Precision: the phase r / lambda reaches thousands of revolutions, so it is formed in FP64 and
// reduced to its fractional part before the sine and cosine.  For complex64 output r comes from
// an FP32 reciprocal square root refined by one FP64 Newton step (relative error ~1e-14), the
// reduced phase goes to the hardware sine/cosine (argument in revolutions) and sums are FP32.
// For complex128 output everything is FP64.
#include "common.hpp"

namespace cgh {
namespace {

constexpr int kTX = 64, kTY = 16, kRows = 4, kThreads = 256;

struct DirectArgs {
    const double4 *pts;
    int64_t n;
    int32_t nx, ny;
    int64_t ox, oy;
    double pitch, inv_lambda, tan2;  // tan2 = tan(theta)^2
    void *out;
    int64_t ld;
};

template <bool CIRC, bool F64>
__global__ __launch_bounds__(kThreads) void direct_kernel(DirectArgs a)
{
    __shared__ double4 sp[kThreads];      // x, y, z^2, amplitude
    __shared__ double sr2[kThreads];      // disk radius^2 (metres^2)
    __shared__ int swave[kThreads / 64];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int col = blockIdx.x * kTX + lane;
    const int row0 = blockIdx.y * kTY + wave;
    const double xh = (double)(a.ox + col) * a.pitch;
    double yh[kRows];
#pragma unroll
    for (int k = 0; k < kRows; k++) yh[k] = (double)(a.oy + row0 + 4 * k) * a.pitch;

    // tile rectangle in metres (pixel centres), for culling
    const double tx0 = (double)(a.ox + (int64_t)blockIdx.x * kTX) * a.pitch;
    const double tx1 = tx0 + (kTX - 1) * a.pitch;
    const double ty0 = (double)(a.oy + (int64_t)blockIdx.y * kTY) * a.pitch;
    const double ty1 = ty0 + (kTY - 1) * a.pitch;

    double accd_re[kRows], accd_im[kRows];
    float accf_re[kRows], accf_im[kRows];
#pragma unroll
    for (int k = 0; k < kRows; k++) {
        accd_re[k] = accd_im[k] = 0.0;
        accf_re[k] = accf_im[k] = 0.0f;
    }

    for (int64_t base = 0; base < a.n; base += kThreads) {
        const int64_t j = base + tid;
        bool keep = false;
        double4 p = make_double4(0, 0, 0, 0);
        double r2 = 0.0;
        if (j < a.n) {
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
            for (int rr = 0; rr < kRows; rr++) {
                const double dy = yh[rr] - q.y;
                const double rho2 = fma(dy, dy, dx2);
                const double d2 = rho2 + q.z;
                if (F64) {
                    double amp = q.w;
                    if (CIRC && !(rho2 < sr2[k])) amp = 0.0;
                    const double t = sqrt(d2) * a.inv_lambda;
                    const double f = t - floor(t);
                    double s, c;
                    sincospi(2.0 * f, &s, &c);
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
        for (int rr = 0; rr < kRows; rr++) {
            const int row = row0 + 4 * rr;
            if (row >= a.ny) continue;
            if (F64) {
                double2 *o = (double2 *)a.out;
                o[(int64_t)row * a.ld + col] = make_double2(accd_re[rr], accd_im[rr]);
            } else {
                float2 *o = (float2 *)a.out;
                o[(int64_t)row * a.ld + col] = make_float2(accf_re[rr], accf_im[rr]);
            }
        }
    }
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
    dim3 grid((nx + kTX - 1) / kTX, (ny + kTY - 1) / kTY);
    if (grid.y > 65535) return fail(CGH_EINVAL, "ny too large");
    const bool f64 = out_dtype == CGH_C128, circ = window == CGH_CIRC;
    ProfScope prof("direct", s);
    if (circ && f64) hipLaunchKernelGGL((direct_kernel<true, true>), grid, dim3(kThreads), 0, s, a);
    else if (circ) hipLaunchKernelGGL((direct_kernel<true, false>), grid, dim3(kThreads), 0, s, a);
    else if (f64) hipLaunchKernelGGL((direct_kernel<false, true>), grid, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL((direct_kernel<false, false>), grid, dim3(kThreads), 0, s, a);
    CGH_CHECK_LAUNCH("direct_kernel");
    return CGH_OK;
}
