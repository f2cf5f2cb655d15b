// Holograms with a coiflet LUT (the wavelet family the paper names, Sec. 2) for gfx950.
//
// A coiflet coefficient reaches beyond its 2^L block, so the tile-local inverse of the Haar path
// does not apply.  Each (sub-)window is grown by a halo of 5 2^L pixels on every side, the points'
// coefficients are superposed into its wavelet field (the same Eq.(2) superposition as for Haar:
// the superposition does not depend on the wavelet), the field is inverted as a whole with the
// periodised synthesis filter bank, level by level (columns then rows, each the transpose of the
// analysis step), and the centre is copied into the hologram.  Pixels of the centre only see
// coefficients whose filters lie inside the grown window, so the result is that of the unbounded
// transform: exact for gamma >= 1.
#include <algorithm>

#include "common.hpp"

namespace cgh {
namespace {

struct SynthFilters {
    float lo[8], hi[8];
    int taps;
};

// x[n] = sum over taps t with t = n (mod 2) of lo[t] a[k] + hi[t] d[k], k = (n - t) / 2 modulo the
// half length: a = the first half of the line, d the second (periodised synthesis).
__device__ inline float2 synth_point(const float2 *line, int64_t step, int n, int len, const SynthFilters &f)
{
    const int half = len / 2;
    float2 acc = make_float2(0.0f, 0.0f);
    for (int t = n & 1; t < f.taps; t += 2) {
        int k = (n - t) / 2;  // n - t is even
        k = k < 0 ? k + half : k;
        const float2 a = line[(int64_t)k * step], d = line[(int64_t)(half + k) * step];
        acc.x += f.lo[t] * a.x + f.hi[t] * d.x;
        acc.y += f.lo[t] * a.y + f.hi[t] * d.y;
    }
    return acc;
}

// Columns (COLS) or rows of the top-left h x w region of `in` (row stride ld) into `out`.
template <bool COLS>
__global__ __launch_bounds__(256) void synth_kernel(const float2 *in, float2 *out, int64_t ld, int h, int w,
                                                    SynthFilters f)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= w) return;
    if (COLS)   // output (row y, column x) from column x
        out[(int64_t)y * ld + x] = synth_point(in + x, ld, y, h, f);
    else        // output (row y, column x) from row y
        out[(int64_t)y * ld + x] = synth_point(in + (int64_t)y * ld, 1, x, w, f);
}

}  // namespace

int coiflet_hologram(const wasabi_lut *lut, const wasabi_point *pts, int64_t n, int64_t ox, int64_t oy,
                     int32_t nx, int32_t ny, int32_t sub, void *u, int64_t ld_u, hipStream_t s)
{
    const int L = lut->L, H = 5 << L;  // the six-tap filters' reach over L levels, < 5 2^L
    if (sub == 0) sub = std::max(nx, ny);
    const int32_t sx = std::min(sub, nx), sy = std::min(sub, ny);
    const int64_t ex = (int64_t)sx + 2 * H, ey = (int64_t)sy + 2 * H;
    if (ex > INT32_MAX || ey > INT32_MAX || ex * ey > (INT64_C(1) << 34))
        return fail(CGH_EINVAL, "sub-hologram of %lld x %lld with its halo is too large", (long long)ex,
                    (long long)ey);
    int rc = prepare_pool();
    if (rc) return rc;
    double lo[8], hi[8];
    SynthFilters f;
    f.taps = wavelet_filters(lut->prm.wavelet, lo, hi);
    for (int t = 0; t < f.taps; ++t) {
        f.lo[t] = (float)lo[t];
        f.hi[t] = (float)hi[t];
    }
    Scratch sc(s);
    float2 *A, *B;
    if ((rc = sc.alloc((void **)&A, sizeof(float2) * (size_t)(ex * ey)))) return rc;
    if ((rc = sc.alloc((void **)&B, sizeof(float2) * (size_t)(ex * ey)))) return rc;
    for (int64_t t0 = 0; t0 < ny; t0 += sub) {
        for (int64_t s0 = 0; s0 < nx; s0 += sub) {
            const int32_t wx = (int32_t)std::min<int64_t>(sub, nx - s0) + 2 * H;
            const int32_t wy = (int32_t)std::min<int64_t>(sub, ny - t0) + 2 * H;
            if ((rc = wasabi_superpose(lut, pts, n, ox + s0 - H, oy + t0 - H, wx, wy, A, 0, s))) return rc;
            {
                ProfScope prof("coiflet_idwt", s);
                for (int l = L - 1; l >= 0; --l) {
                    const int h = wy >> l, w = wx >> l;
                    const dim3 grid((unsigned)((w + 255) / 256), (unsigned)h);
                    hipLaunchKernelGGL(synth_kernel<true>, grid, dim3(256), 0, s, A, B, (int64_t)wx, h, w, f);
                    hipLaunchKernelGGL(synth_kernel<false>, grid, dim3(256), 0, s, B, A, (int64_t)wx, h, w, f);
                }
                CGH_CHECK_LAUNCH("synth_kernel");
            }
            CGH_TRY_HIP(hipMemcpy2DAsync((float2 *)u + t0 * ld_u + s0, sizeof(float2) * ld_u,
                                         A + (int64_t)H * wx + H, sizeof(float2) * wx,
                                         sizeof(float2) * (wx - 2 * H), wy - 2 * H, hipMemcpyDeviceToDevice, s));
        }
    }
    return CGH_OK;
}

}  // namespace cgh
