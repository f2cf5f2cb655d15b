// Angular-spectrum propagation of a sampled complex field (the numerical reconstruction the paper
// assesses holograms by, Sec. 3) and the hologram through a wavefront recording plane (the method the
// conclusion names as the next step) for gfx950.
//
// u' = IFFT2(FFT2(u) H), H(fx, fy) = exp(i 2 pi d sqrt(1/lambda^2 - fx^2 - fy^2)) on the propagating
// disk and 0 beyond it.  The 2-D transforms are radix-2 FFTs of whole rows in LDS, one workgroup per
// row, with 64 x 64 tiled transposes between the passes:
//   1. forward FFT of every row of u into A;
//   2. A (ny x nx) transposed into B (nx x ny): row kx of B is the column of spatial frequency fx;
//   3. per row of B: forward FFT along y, times H(fx, fy), inverse FFT along y;
//   4. B transposed back into A;
//   5. inverse FFT of every row of A into u'.
// Every pass reads and writes the field once (16 B per pixel); the row transforms go two radix-2
// stages per barrier; twiddles and the transfer
// function's phase come from FP64 angles (the phase reduced to revolutions first), rounded to FP32.
#include <cmath>

#include "common.hpp"

namespace cgh {
// wasabi_quantize with every depth first reduced by z_shift (lut.hip).
int quantize_shifted(const wasabi_lut *lut, const double *pts, int64_t n, double z_shift,
                     wasabi_point *out, hipStream_t s);

namespace {

constexpr int kFftThreads = 256;
constexpr int kMaxFft = 8192;   // row length: the row (64 KiB of complex64) lives in LDS

// w[k] = exp(-2 pi i k / n), 0 <= k < n / 2.
__global__ void twiddle_kernel(float2 *w, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n / 2) return;
    double s, c;
    sincospi(-2.0 * (double)k / (double)n, &s, &c);
    w[k] = make_float2((float)c, (float)s);
}

__device__ inline float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline int bit_reverse(int i, int logn) { return (int)(__brev((unsigned)i) >> (32 - logn)); }

// Decimation-in-time FFT of buf[0, n) in LDS, input in bit-reversed order, output in natural order.
// The radix-2 stages go two at a time: a thread loads the four points i0 + {0, h, 2h, 3h} of a
// block of 4h, does the stage of span h and the stage of span 2h on them in registers and stores
// them back, so there is one barrier and one LDS round trip per two stages; an odd last stage is
// plain radix 2.  INV: the conjugate twiddles (no 1/n).
template <bool INV>
__device__ inline float2 twiddle(const float2 *tw, int k)
{
    float2 w = tw[k];
    if (INV) w.y = -w.y;
    return w;
}

template <bool INV>
__device__ inline void fft_lds(float2 *buf, int n, int logn, const float2 *tw)
{
    int s = 1;
    for (; s + 1 <= logn; s += 2) {
        const int h = 1 << (s - 1);            // span of the first of the two stages
        const int st1 = n >> s, st2 = n >> (s + 1);  // twiddle strides: W_2h^j = tw[j n / 2h]
        for (int b = threadIdx.x; b < n / 4; b += blockDim.x) {
            const int j = b & (h - 1);
            const int i0 = ((b >> (s - 1)) << (s + 1)) + j;
            const float2 w1 = twiddle<INV>(tw, j * st1);
            const float2 w2 = twiddle<INV>(tw, j * st2), w3 = twiddle<INV>(tw, (j + h) * st2);
            const float2 a0 = buf[i0], a1 = buf[i0 + h], a2 = buf[i0 + 2 * h], a3 = buf[i0 + 3 * h];
            const float2 t1 = cmul(w1, a1), t3 = cmul(w1, a3);
            const float2 b0 = make_float2(a0.x + t1.x, a0.y + t1.y), b1 = make_float2(a0.x - t1.x, a0.y - t1.y);
            const float2 b2 = make_float2(a2.x + t3.x, a2.y + t3.y), b3 = make_float2(a2.x - t3.x, a2.y - t3.y);
            const float2 u2 = cmul(w2, b2), u3 = cmul(w3, b3);
            buf[i0] = make_float2(b0.x + u2.x, b0.y + u2.y);
            buf[i0 + 2 * h] = make_float2(b0.x - u2.x, b0.y - u2.y);
            buf[i0 + h] = make_float2(b1.x + u3.x, b1.y + u3.y);
            buf[i0 + 3 * h] = make_float2(b1.x - u3.x, b1.y - u3.y);
        }
        __syncthreads();
    }
    if (s == logn) {  // one radix-2 stage left
        const int h = 1 << (s - 1), stride = n >> s;
        for (int b = threadIdx.x; b < n / 2; b += blockDim.x) {
            const int j = b & (h - 1);
            const int i0 = ((b >> (s - 1)) << s) + j, i1 = i0 + h;
            const float2 a = buf[i0], t = cmul(twiddle<INV>(tw, j * stride), buf[i1]);
            buf[i0] = make_float2(a.x + t.x, a.y + t.y);
            buf[i1] = make_float2(a.x - t.x, a.y - t.y);
        }
        __syncthreads();
    }
}

// Row r of `in` (row stride ld_in) -> FFT -> times `scale` -> row r of `out` (row stride ld_out).
template <bool INV>
__global__ __launch_bounds__(kFftThreads) void fft_rows_kernel(const float2 *in, int64_t ld_in, float2 *out,
                                                               int64_t ld_out, int n, int logn,
                                                               const float2 *tw, float scale)
{
    extern __shared__ float2 buf[];
    const float2 *src = in + (int64_t)blockIdx.x * ld_in;
    for (int i = threadIdx.x; i < n; i += blockDim.x) buf[bit_reverse(i, logn)] = src[i];
    __syncthreads();
    fft_lds<INV>(buf, n, logn, tw);
    float2 *dst = out + (int64_t)blockIdx.x * ld_out;
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = make_float2(buf[i].x * scale, buf[i].y * scale);
}

// Row kx of the transposed spectrum (nx rows of ny): forward FFT along y, times H(fx, fy), inverse
// FFT along y, times 1/ny, in place.
__global__ __launch_bounds__(kFftThreads) void column_transfer_kernel(float2 *data, int nx, int ny, int logny,
                                                                      const float2 *tw, double fx_unit,
                                                                      double fy_unit, double inv_lambda2,
                                                                      double distance)
{
    extern __shared__ float2 buf[];
    const int kx = blockIdx.x;
    float2 *row = data + (int64_t)kx * ny;
    for (int i = threadIdx.x; i < ny; i += blockDim.x) buf[bit_reverse(i, logny)] = row[i];
    __syncthreads();
    fft_lds<false>(buf, ny, logny, tw);
    const double fx = (double)(kx < nx / 2 ? kx : kx - nx) * fx_unit;
    const float scale = 1.0f / (float)ny;
    for (int ky = threadIdx.x; ky < ny; ky += blockDim.x) {
        const double fy = (double)(ky < ny / 2 ? ky : ky - ny) * fy_unit;
        const double arg = inv_lambda2 - fx * fx - fy * fy;
        float2 h = make_float2(0.0f, 0.0f);
        if (arg > 0.0) {
            const double rev = distance * sqrt(arg);  // revolutions; whole ones dropped
            double s, c;
            sincospi(2.0 * (rev - floor(rev)), &s, &c);
            h = make_float2((float)c * scale, (float)s * scale);
        }
        buf[ky] = cmul(buf[ky], h);
    }
    __syncthreads();
    // natural -> bit-reversed order for the inverse transform (each pair swapped once)
    for (int i = threadIdx.x; i < ny; i += blockDim.x) {
        const int r = bit_reverse(i, logny);
        if (i < r) {
            const float2 t = buf[i];
            buf[i] = buf[r];
            buf[r] = t;
        }
    }
    __syncthreads();
    fft_lds<true>(buf, ny, logny, tw);
    for (int i = threadIdx.x; i < ny; i += blockDim.x) row[i] = buf[i];
}

// out (cols x rows) = transpose of in (rows x cols), both contiguous; 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void transpose_kernel(const float2 *in, float2 *out, int rows, int cols)
{
    __shared__ float2 t[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    for (int r = ty; r < 64; r += 4)
        if (r0 + r < rows && c0 + tx < cols) t[r][tx] = in[(r0 + r) * cols + c0 + tx];
    __syncthreads();
    for (int c = ty; c < 64; c += 4)
        if (c0 + c < cols && r0 + tx < rows) out[(c0 + c) * rows + r0 + tx] = t[tx][c];
}

int log2_exact(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return (1 << l) == n ? l : -1;
}

}  // namespace

int propagate_impl(const void *u_in, void *u_out, int32_t nx, int32_t ny, double distance, double pitch,
                   double wavelength, hipStream_t s)
{
    if (!u_in || !u_out) return fail(CGH_EINVAL, "NULL field");
    const int lx = log2_exact(nx), ly = log2_exact(ny);
    if (lx < 6 || ly < 6 || nx > kMaxFft || ny > kMaxFft)
        return fail(CGH_EINVAL, "field %d x %d: sides must be powers of two in [64, %d]", nx, ny, kMaxFft);
    if (!(pitch > 0) || !(wavelength > 0) || !std::isfinite(distance) || !std::isfinite(pitch) ||
        !std::isfinite(wavelength))
        return fail(CGH_EINVAL, "need pitch > 0, wavelength > 0 and a finite distance");
    int rc = prepare_pool();
    if (rc) return rc;
    Scratch sc(s);
    float2 *A, *B, *twx, *twy;
    const size_t field = sizeof(float2) * (size_t)nx * ny;
    if ((rc = sc.alloc((void **)&A, field))) return rc;
    if ((rc = sc.alloc((void **)&B, field))) return rc;
    if ((rc = sc.alloc((void **)&twx, sizeof(float2) * (nx / 2)))) return rc;
    if ((rc = sc.alloc((void **)&twy, sizeof(float2) * (ny / 2)))) return rc;
    ProfScope prof("propagate", s);
    hipLaunchKernelGGL(twiddle_kernel, dim3((nx / 2 + 255) / 256), dim3(256), 0, s, twx, nx);
    hipLaunchKernelGGL(twiddle_kernel, dim3((ny / 2 + 255) / 256), dim3(256), 0, s, twy, ny);
    CGH_CHECK_LAUNCH("twiddle_kernel");
    hipLaunchKernelGGL(fft_rows_kernel<false>, dim3(ny), dim3(kFftThreads), sizeof(float2) * nx, s,
                       (const float2 *)u_in, (int64_t)nx, A, (int64_t)nx, nx, lx, twx, 1.0f);
    CGH_CHECK_LAUNCH("fft_rows_kernel");
    hipLaunchKernelGGL(transpose_kernel, dim3(nx / 64, ny / 64), dim3(256), 0, s, A, B, ny, nx);
    CGH_CHECK_LAUNCH("transpose_kernel");
    hipLaunchKernelGGL(column_transfer_kernel, dim3(nx), dim3(kFftThreads), sizeof(float2) * ny, s, B, nx,
                       ny, ly, twy, 1.0 / ((double)nx * pitch), 1.0 / ((double)ny * pitch),
                       1.0 / (wavelength * wavelength), distance);
    CGH_CHECK_LAUNCH("column_transfer_kernel");
    hipLaunchKernelGGL(transpose_kernel, dim3(ny / 64, nx / 64), dim3(256), 0, s, B, A, nx, ny);
    CGH_CHECK_LAUNCH("transpose_kernel");
    hipLaunchKernelGGL(fft_rows_kernel<true>, dim3(ny), dim3(kFftThreads), sizeof(float2) * nx, s,
                       (const float2 *)A, (int64_t)nx, (float2 *)u_out, (int64_t)nx, nx, lx, twx,
                       1.0f / (float)nx);
    CGH_CHECK_LAUNCH("fft_rows_kernel");
    return CGH_OK;
}

}  // namespace cgh

extern "C" int cgh_propagate(const void *u_in, void *u_out, int32_t nx, int32_t ny, double distance,
                             double pitch, double wavelength, void *stream)
{
    return cgh::propagate_impl(u_in, u_out, nx, ny, distance, pitch, wavelength, (hipStream_t)stream);
}

extern "C" int wasabi_hologram_wrp(const wasabi_lut *lut, const double *pts, int64_t n, double z_wrp,
                                   int32_t nx, int32_t ny, void *u, void *stream)
{
    using namespace cgh;
    if (!lut) return fail(CGH_EINVAL, "lut is NULL");
    if (n < 0 || n > INT32_MAX) return fail(CGH_EINVAL, "n out of range");
    if (n > 0 && !pts) return fail(CGH_EINVAL, "pts is NULL");
    if (!u) return fail(CGH_EINVAL, "u is NULL");
    if (!std::isfinite(z_wrp)) return fail(CGH_EINVAL, "z_wrp must be finite");
    const int lx = log2_exact(nx), ly = log2_exact(ny);
    if (lx < 6 || ly < 6 || nx > kMaxFft || ny > kMaxFft)
        return fail(CGH_EINVAL, "hologram %d x %d: sides must be powers of two in [64, %d]", nx, ny, kMaxFft);
    hipStream_t s = (hipStream_t)stream;
    int rc = prepare_pool();
    if (rc) return rc;
    Scratch sc(s);
    wasabi_point *q = nullptr;
    if (n > 0 && (rc = sc.alloc((void **)&q, sizeof(wasabi_point) * (size_t)n))) return rc;
    if (n > 0 && (rc = quantize_shifted(lut, pts, n, z_wrp, q, s))) return rc;
    rc = lut->prm.wavelet == CGH_HAAR ? wasabi_hologram_fused(lut, q, n, 0, 0, nx, ny, u, nx, s)
                                      : wasabi_hologram(lut, q, n, 0, 0, nx, ny, 0, u, nx, s);
    if (rc) return rc;
    return propagate_impl(u, u, nx, ny, z_wrp, lut->prm.pitch, lut->prm.wavelength, s);
}
