// Coefficient LUT of the wavelet path (Sec. 2, step 1: pre-computation) and point quantisation.
//
//  psf_haar_kernel : PSF table  exp(i 2 pi r / lambda) circ()  sampled in FP64 and transformed
//                    by an L-level orthonormal Haar transform, one aligned 2^L x 2^L block at a
//                    time in LDS (Haar blocks are independent, so no halo is needed).
//  select_kernel   : per plane, the N_r strongest coefficients.  Strength is |c|^2 (FP64)
//                    rounded to FP32, so coefficients equal in exact arithmetic (the PSF's
//                    transposed twins) compare equal; equal strengths go to the lower flat table
//                    index.  A 4-pass MSB radix select finds the threshold strength, a second
//                    radix select over flat indices splits the tie at the threshold, and an
//                    order-preserving compaction writes (value, key) entries grouped by Haar
//                    block plus the per-block offsets.
//  quantize_kernel : points (metres) -> grid position and plane index.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "common.hpp"

namespace cgh {
namespace {

// ---- round-to-nearest-even conversions from FP64, written from the IEEE 754 encodings --------
__host__ __device__ inline uint32_t f64_to_small_float(double v, int mant_bits, int exp_bias,
                                                       int exp_max_field)
{
    uint64_t b;
    memcpy(&b, &v, 8);
    const uint32_t sign = (uint32_t)(b >> 63) << (mant_bits + (exp_max_field == 31 ? 5 : 8));
    const int ebits = (exp_max_field == 31) ? 5 : 8;
    const uint32_t inf = ((1u << ebits) - 1u) << mant_bits;
    const int dexp = (int)((b >> 52) & 0x7ff);
    const uint64_t dman = b & ((UINT64_C(1) << 52) - 1);
    if (dexp == 0x7ff) return sign | inf | (dman ? (1u << (mant_bits - 1)) : 0u);
    if (dexp == 0) return sign;  // FP64 subnormals are far below the target's range
    const int e = dexp - 1023;   // value = 1.f * 2^e
    const int emin = 1 - exp_bias;
    if (e > exp_bias) return sign | inf;
    if (e < emin - mant_bits - 1) return sign;  // below half the smallest subnormal
    const uint64_t sig = (UINT64_C(1) << 52) | dman;
    const int shift = 52 - mant_bits + (e < emin ? emin - e : 0);
    uint64_t q = sig >> shift;
    const uint64_t rem = sig & ((UINT64_C(1) << shift) - 1);
    const uint64_t half = UINT64_C(1) << (shift - 1);
    if (rem > half || (rem == half && (q & 1))) q++;
    if (e < emin) return sign | (uint32_t)q;  // subnormal (q == 2^mant_bits -> smallest normal)
    int fe = e + exp_bias;
    if (q >> (mant_bits + 1)) {
        q >>= 1;
        fe++;
    }
    if (fe >= (1 << ebits) - 1) return sign | inf;
    return sign | ((uint32_t)fe << mant_bits) | ((uint32_t)q & ((1u << mant_bits) - 1));
}

__host__ __device__ inline uint32_t f64_to_f16_bits(double v) { return f64_to_small_float(v, 10, 15, 31); }
__host__ __device__ inline uint32_t f64_to_bf16_bits(double v) { return f64_to_small_float(v, 7, 127, 255); }

inline double f16_bits_to_f64(uint32_t h)
{
    const int e = (h >> 10) & 31, m = h & 1023;
    double v = (e == 0) ? std::ldexp((double)m, -24)
                        : (e == 31 ? (m ? NAN : INFINITY) : std::ldexp((double)(m | 1024), e - 25));
    return (h & 0x8000) ? -v : v;
}

inline double bf16_bits_to_f64(uint32_t h)
{
    const uint32_t f = h << 16;
    float x;
    memcpy(&x, &f, 4);
    return (double)x;
}

// (block row, block column, in-block code) -> flat index row * W + col of the plane's
// Mallat-layout table.
__host__ __device__ inline int64_t block_to_flat(int br, int bc, int code, int W, int L)
{
    const int B = 1 << L;
    const int ir = code / B, ic = code % B;
    int lev = L, band = 0, mm = ir, nn = ic;
    for (int l = 1; l <= L; ++l) {
        const int h = B >> l;
        if (ir >= h || ic >= h) {
            lev = l;
            band = 2 * (ir >= h) + (ic >= h);
            mm = ir - (ir >= h ? h : 0);
            nn = ic - (ic >= h ? h : 0);
            break;
        }
    }
    const int h = B >> lev, s = W >> lev;
    const int64_t row = ((band & 2) ? s : 0) + (int64_t)br * h + mm;
    const int64_t col = ((band & 1) ? s : 0) + (int64_t)bc * h + nn;
    return row * W + col;
}

// ---- PSF table + in-block forward Haar ------------------------------------------------------
// The disk's centre is (W/2 + sx, W/2 + sy): sx = sy = 0 but for phase tables.
template <int L>
__global__ __launch_bounds__(256) void psf_haar_kernel(int W, int nb, int sx, int sy, double z,
                                                       double R2, double pitch, double lambda,
                                                       double2 *coef, uint32_t *magq)
{
    constexpr int B = 1 << L, BB = B * B;
    constexpr int G = BB >= 256 ? 1 : 256 / BB;  // blocks per workgroup
    constexpr int NPIX = G * BB;
    constexpr int MAXQ = (NPIX / 4 + 255) / 256;
    __shared__ double2 buf[NPIX];
    const int c = W / 2;
    const int64_t nblk = (int64_t)nb * nb;
    const int64_t blk0 = (int64_t)blockIdx.x * G;

    for (int p = threadIdx.x; p < NPIX; p += 256) {
        const int g = p / BB, code = p % BB;
        const int64_t blk = blk0 + g;
        double2 v = make_double2(0.0, 0.0);
        if (blk < nblk) {
            const int br = (int)(blk / nb), bc = (int)(blk % nb);
            const double dr = (double)(br * B + code / B - c - sy);
            const double dq = (double)(bc * B + code % B - c - sx);
            if (dq * dq + dr * dr < R2) {
                const double dist = sqrt((dq * pitch) * (dq * pitch) + (dr * pitch) * (dr * pitch) + z * z);
                const double t = dist / lambda;  // revolutions; whole ones dropped below
                double s, cs;
                sincospi(2.0 * (t - floor(t)), &s, &cs);
                v = make_double2(cs, s);
            }
        }
        buf[p] = v;
    }
    __syncthreads();

    for (int l = 1; l <= L; ++l) {
        const int h2 = B >> l;
        const int per = h2 * h2, nq = G * per;
        double2 S[MAXQ], H[MAXQ], V[MAXQ], D[MAXQ];
#pragma unroll
        for (int k = 0; k < MAXQ; ++k) {
            const int qi = threadIdx.x + 256 * k;
            if (qi < nq) {
                const int g = qi / per, m = (qi % per) / h2, n = qi % h2;
                const double2 *blkp = buf + g * BB;
                const double2 a = blkp[(2 * m) * B + 2 * n], b = blkp[(2 * m) * B + 2 * n + 1];
                const double2 cc = blkp[(2 * m + 1) * B + 2 * n], d = blkp[(2 * m + 1) * B + 2 * n + 1];
                S[k] = make_double2((a.x + b.x + cc.x + d.x) * 0.5, (a.y + b.y + cc.y + d.y) * 0.5);
                H[k] = make_double2((a.x - b.x + cc.x - d.x) * 0.5, (a.y - b.y + cc.y - d.y) * 0.5);
                V[k] = make_double2((a.x + b.x - cc.x - d.x) * 0.5, (a.y + b.y - cc.y - d.y) * 0.5);
                D[k] = make_double2((a.x - b.x - cc.x + d.x) * 0.5, (a.y - b.y - cc.y + d.y) * 0.5);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < MAXQ; ++k) {
            const int qi = threadIdx.x + 256 * k;
            if (qi < nq) {
                const int g = qi / per, m = (qi % per) / h2, n = qi % h2;
                double2 *blkp = buf + g * BB;
                blkp[m * B + n] = S[k];
                blkp[m * B + h2 + n] = H[k];
                blkp[(h2 + m) * B + n] = V[k];
                blkp[(h2 + m) * B + h2 + n] = D[k];
            }
        }
        __syncthreads();
    }

    for (int p = threadIdx.x; p < NPIX; p += 256) {
        const int64_t blk = blk0 + p / BB;
        if (blk < nblk) {
            const double2 v = buf[p];
            const int64_t at = blk * BB + p % BB;
            coef[at] = v;
            // strength key: |c|^2 rounded to FP32 (non-negative, so its bits order like its value)
            magq[at] = __float_as_uint((float)(v.x * v.x + v.y * v.y));
        }
    }
}

// ---- coiflet tables: PSF in the pixel layout, periodised filter-bank transform, block order -----
struct DwtFilters {
    double lo[8], hi[8];
    int taps;
};

// The W x W PSF table, disk centred on (W/2 + sx, W/2 + sy), row-major.
__global__ __launch_bounds__(256) void psf_fill_kernel(int W, int sx, int sy, double z, double R2,
                                                       double pitch, double lambda, double2 *T)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)W * W) return;
    const int c = W / 2;
    const double dr = (double)((int)(i / W) - c - sy), dq = (double)((int)(i % W) - c - sx);
    double2 v = make_double2(0.0, 0.0);
    if (dq * dq + dr * dr < R2) {
        const double dist = sqrt((dq * pitch) * (dq * pitch) + (dr * pitch) * (dr * pitch) + z * z);
        const double t = dist / lambda;  // revolutions; whole ones dropped below
        double sn, cs;
        sincospi(2.0 * (t - floor(t)), &sn, &cs);
        v = make_double2(cs, sn);
    }
    T[i] = v;
}

// One periodised analysis step on every row (ROWS) or column of the top-left h x w region of a
// W-wide table: a[k] = sum_t lo[t] x[(2k + t) mod len], d[k] = sum_t hi[t] x[(2k + t) mod len],
// a into the first half of the line, d into the second.  One workgroup per line, staged in LDS.
template <bool ROWS>
__global__ __launch_bounds__(256) void dwt_line_kernel(double2 *T, int W, int h, int w, DwtFilters f)
{
    extern __shared__ double2 line[];
    const int len = ROWS ? w : h, half = len / 2;
    const int64_t base = ROWS ? (int64_t)blockIdx.x * W : (int64_t)blockIdx.x;
    const int64_t step = ROWS ? 1 : W;
    for (int i = threadIdx.x; i < len; i += blockDim.x) line[i] = T[base + i * step];
    __syncthreads();
    for (int k = threadIdx.x; k < half; k += blockDim.x) {
        double2 a = make_double2(0.0, 0.0), d = make_double2(0.0, 0.0);
        for (int t = 0; t < f.taps; ++t) {
            const double2 x = line[(2 * k + t) % len];
            a.x += f.lo[t] * x.x;
            a.y += f.lo[t] * x.y;
            d.x += f.hi[t] * x.x;
            d.y += f.hi[t] * x.y;
        }
        T[base + k * step] = a;
        T[base + (half + k) * step] = d;
    }
}

// Mallat-layout coefficients -> the block-major order of the selection (block (br, bc), code) and
// their strength keys, as psf_haar_kernel writes them.
__global__ __launch_bounds__(256) void mallat_to_blocks_kernel(const double2 *T, int W, int L, double2 *coef,
                                                               uint32_t *magq)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)W * W) return;
    const int BB = 1 << (2 * L), nb = W >> L;
    const int64_t blk = i / BB;
    const double2 v = T[block_to_flat((int)(blk / nb), (int)(blk % nb), (int)(i % BB), W, L)];
    coef[i] = v;
    magq[i] = __float_as_uint((float)(v.x * v.x + v.y * v.y));
}

// ---- block-wide exclusive scan of one flag per thread (1024 threads) --------------------------
__device__ inline int block_excl_count(bool flag, int *wave_tot, int &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t m = __ballot(flag);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wave] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        const int t = wave_tot[w];
        off += (w < wave) ? t : 0;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return off + before;
}

// ---- per-plane selection of the N_r largest magnitudes -------------------------------------
struct SelPlane {
    int64_t coef_off;     // first coefficient of the plane in coef / mag2
    int64_t count;        // W * W
    int64_t nr;           // entries to keep
    int64_t entry_base;   // first output entry
    int64_t blkoff_base;  // first element of the plane's block offsets
    int32_t nb;
    int32_t pad;
};

template <int VT>
__global__ __launch_bounds__(1024) void select_kernel(const double2 *coef_all, const uint32_t *magq_all,
                                                      const SelPlane *planes, int L,
                                                      void *values_all, uint16_t *keys_all,
                                                      int32_t *blk_off_all)
{
    const SelPlane pl = planes[blockIdx.x];
    const double2 *coef = coef_all + pl.coef_off;
    const uint32_t *mq = magq_all + pl.coef_off;
    const int64_t count = pl.count, nr = pl.nr;
    const int nb = pl.nb, W = nb << L;
    uint16_t *keys = keys_all + pl.entry_base;
    int32_t *blk_off = blk_off_all + pl.blkoff_base;
    void *values = (char *)values_all + (VT == CGH_F32 ? 8 : 4) * pl.entry_base;
    const int BB = 1 << (2 * L);
    const int BS = block_stride(L);
    __shared__ uint32_t hist[256];
    __shared__ int wave_tot[16];
    __shared__ int s_digit;
    __shared__ long long s_k, s_ties;

    // (1) MSB-first radix select on the strength keys: `thr` is the key of the nr-th strongest
    //     coefficient, `need` how many coefficients with key == thr are kept, `ties` how many
    //     have key == thr.
    uint32_t prefix = 0, mask = 0;
    long long k = nr;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (int i = threadIdx.x; i < 256; i += 1024) hist[i] = 0;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < count; i += 1024) {
            const uint32_t b = mq[i];
            if ((b & mask) == prefix) atomicAdd(&hist[(b >> shift) & 255], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            long long cum = 0;
            int v = 255;
            for (; v > 0; --v) {
                if (cum + (long long)hist[v] >= k) break;
                cum += hist[v];
            }
            s_digit = v;
            s_k = k - cum;
            s_ties = hist[v];
        }
        __syncthreads();
        prefix |= (uint32_t)s_digit << shift;
        mask |= 0xffu << shift;
        k = s_k;
        __syncthreads();
    }
    const uint32_t thr = prefix;
    const long long need = k, ties = s_ties;

    // (2) equal strengths go to the lower flat table index: `fthr` is the need-th smallest flat
    //     index among the tied coefficients (radix select from the low end).
    uint32_t fthr = 0xffffffffu;
    if (need < ties) {
        uint32_t fp = 0, fm = 0;
        long long kk = need;
        for (int pass = 0; pass < 4; ++pass) {
            const int shift = 24 - 8 * pass;
            for (int i = threadIdx.x; i < 256; i += 1024) hist[i] = 0;
            __syncthreads();
            for (int64_t i = threadIdx.x; i < count; i += 1024) {
                if (mq[i] != thr) continue;
                const int64_t blk = i / BB;
                const uint32_t f = (uint32_t)block_to_flat((int)(blk / nb), (int)(blk % nb), (int)(i % BB), W, L);
                if ((f & fm) == fp) atomicAdd(&hist[(f >> shift) & 255], 1u);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                long long cum = 0;
                int v = 0;
                for (; v < 255; ++v) {
                    if (cum + (long long)hist[v] >= kk) break;
                    cum += hist[v];
                }
                s_digit = v;
                s_k = kk - cum;
            }
            __syncthreads();
            fp |= (uint32_t)s_digit << shift;
            fm |= 0xffu << shift;
            kk = s_k;
            __syncthreads();
        }
        fthr = fp;
    }

    // (3) order-preserving compaction into (value, key) entries grouped by Haar block
    long long running = 0;
    for (int64_t base = 0; base < count; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const bool valid = i < count;
        const uint32_t b = valid ? mq[i] : 0;
        bool take = valid && b > thr;
        if (valid && b == thr) {
            if (need >= ties) {
                take = true;
            } else {
                const int64_t blk = i / BB;
                take = (uint32_t)block_to_flat((int)(blk / nb), (int)(blk % nb), (int)(i % BB), W, L) <= fthr;
            }
        }
        int sel_total;
        const int sel_before = block_excl_count(take, wave_tot, sel_total);
        const long long pos = running + sel_before;
        if (valid && (i % BB) == 0) blk_off[i / BB] = (int32_t)pos;
        if (take && pos < nr) {
            const double2 v = coef[i];
            const int64_t blk = i / BB;
            const int code = (int)(i % BB);
            keys[pos] = (uint16_t)((blk % nb) * BS + code);
            if (VT == CGH_F32) {
                ((float2 *)values)[pos] = make_float2((float)v.x, (float)v.y);
            } else if (VT == CGH_F16) {
                ((uint32_t *)values)[pos] = f64_to_f16_bits(v.x) | (f64_to_f16_bits(v.y) << 16);
            } else {
                ((uint32_t *)values)[pos] = f64_to_bf16_bits(v.x) | (f64_to_bf16_bits(v.y) << 16);
            }
        }
        running += sel_total;
    }
    if (threadIdx.x == 0) blk_off[count / BB] = (int32_t)running;
}

// ---- largest stored |re| / |im| per plane (one workgroup per plane) -------------------------
template <int VT>
__global__ __launch_bounds__(256) void plane_cmax_kernel(const void *values, const int64_t *entry_off,
                                                         float *cmax)
{
    __shared__ float red[256];
    const int64_t e0 = entry_off[blockIdx.x], e1 = entry_off[blockIdx.x + 1];
    float m = 0.0f;
    for (int64_t i = e0 + threadIdx.x; i < e1; i += 256) {
        float re, im;
        if (VT == CGH_F32) {
            const float2 v = ((const float2 *)values)[i];
            re = v.x;
            im = v.y;
        } else {
            const uint32_t w = ((const uint32_t *)values)[i];
            if (VT == CGH_F16) {
                _Float16 lo, hi;
                const uint16_t l16 = (uint16_t)(w & 0xffff), h16 = (uint16_t)(w >> 16);
                __builtin_memcpy(&lo, &l16, 2);
                __builtin_memcpy(&hi, &h16, 2);
                re = (float)lo;
                im = (float)hi;
            } else {
                re = __uint_as_float(w << 16);
                im = __uint_as_float(w & 0xffff0000u);
            }
        }
        m = fmaxf(m, fmaxf(fabsf(re), fabsf(im)));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) cmax[blockIdx.x] = red[0];
}

// ---- dense layout: scatter the kept entries of one table block row into its whole blocks ------
struct DenseJob {
    int64_t entry_base, blkoff_base, dense_base;
    int32_t nb, br, lo, hi, off, pad;
};

__global__ __launch_bounds__(256) void dense_scatter_kernel(const DenseJob *jobs, int L, int vbytes,
                                                            const int32_t *blk_off, const uint16_t *keys,
                                                            const void *values, void *dense)
{
    const DenseJob j = jobs[blockIdx.x];
    const int BB = 1 << (2 * L), BS = block_stride(L);
    const int32_t *bo = blk_off + j.blkoff_base + (int64_t)j.br * j.nb;
    const int32_t e0 = bo[j.lo], e1 = bo[j.hi];
    for (int32_t e = e0 + threadIdx.x; e < e1; e += 256) {
        const int key = keys[j.entry_base + e];
        const int bcol = key / BS, code = key - (key / BS) * BS;
        const int64_t at = j.dense_base + j.off + (int64_t)(bcol - j.lo) * BB + code;
        if (vbytes == 8) ((float2 *)dense)[at] = ((const float2 *)values)[j.entry_base + e];
        else ((uint32_t *)dense)[at] = ((const uint32_t *)values)[j.entry_base + e];
    }
}

// ---- sparse layout: every entry's byte offset in the tile buffer (one workgroup per table) -------
__global__ __launch_bounds__(256) void wide_key_kernel(const DepthDesc *desc, const int32_t *blk_off,
                                                       const uint16_t *keys, int row_words, int32_t *wkeys)
{
    const DepthDesc d = desc[blockIdx.x];
    const int32_t *bo = blk_off + d.blkoff_base;
    for (int br = 0; br < d.nb; ++br) {
        const int32_t e0 = bo[(int64_t)br * d.nb], e1 = bo[(int64_t)(br + 1) * d.nb];
        for (int32_t e = e0 + threadIdx.x; e < e1; e += 256)
            wkeys[d.entry_base + e] = (br * row_words + (int)keys[d.entry_base + e]) * 8;
    }
}

// ---- quantisation ---------------------------------------------------------------------------
// z_shift: subtracted from every depth first (0, or a wavefront recording plane's distance).
__global__ void quantize_kernel(const double4 *pts, int64_t n, double pitch, double z_min,
                                double z_max, double dz, int n_depth, int L, int phases,
                                double z_shift, wasabi_point *out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double4 p = pts[j];
    p.z -= z_shift;
    wasabi_point q;
    q.x = 0;
    q.y = 0;
    q.depth = -1;
    q.a = (float)p.w;
    const double B = phases ? 1.0 : (double)(1 << L);  // snapping grid: 2^L, or the pixel
    if (isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(p.w) && p.z >= z_min &&
        p.z <= z_max) {
        const double sx = B * floor(p.x / pitch / B + 0.5);
        const double sy = B * floor(p.y / pitch / B + 0.5);
        if (fabs(sx) < 1073741824.0 && fabs(sy) < 1073741824.0) {
            int d = (int)floor((p.z - z_min) / dz);
            if (d > n_depth - 1) d = n_depth - 1;
            q.x = (int32_t)sx;
            q.y = (int32_t)sy;
            if (phases) {  // the table of the point's position inside its 2^L block
                const int px = q.x & ((1 << L) - 1), py = q.y & ((1 << L) - 1);
                d = (d << (2 * L)) + (py << L) + px;
            }
            q.depth = d;
        }
    }
    out[j] = q;
}

// ---- canonical <-> internal index maps (host) -------------------------------------------------
// flat index of the plane's Mallat-layout table -> (block row, block column, in-block code)
void flat_to_block(int64_t flat, int W, int L, int &br, int &bc, int &code)
{
    const int B = 1 << L;
    const int row = (int)(flat / W), col = (int)(flat % W);
    int lev = L, band = 0, m = row, n = col;
    for (int l = 1; l <= L; ++l) {
        const int s = W >> l;
        if (row >= s || col >= s) {
            lev = l;
            band = 2 * (row >= s) + (col >= s);
            m = row - (row >= s ? s : 0);
            n = col - (col >= s ? s : 0);
            break;
        }
    }
    const int h = B >> lev;  // band size inside one block
    br = m / h;
    bc = n / h;
    const int ir = ((band & 2) ? h : 0) + m % h;
    const int ic = ((band & 1) ? h : 0) + n % h;
    code = ir * B + ic;
}

size_t value_bytes(int vt) { return vt == CGH_F32 ? 8 : 4; }

// Dense layout for large gamma: row spans from the block offsets, then a scatter kernel.
int build_dense(wasabi_lut *lut, const std::vector<int32_t> &blk_off_host)
{
    const int n = lut->n_tables, B = lut->B, BB = B * B;
    lut->dense = lut->prm.gamma >= kDenseGamma;
    if (!lut->dense) return CGH_OK;
    std::vector<DenseRow> rows;
    std::vector<DenseJob> jobs;
    int64_t total = 0;
    for (int d = 0; d < n; ++d) {
        DepthDesc &dd = lut->desc_host[d];
        const int nb = dd.nb;
        const int32_t *bo = blk_off_host.data() + dd.blkoff_base;
        dd.dense_base = total;
        dd.rows_base = (int64_t)rows.size();
        int64_t off = 0;
        for (int br = 0; br < nb; ++br) {
            int lo = nb, hi = 0;
            for (int bc = 0; bc < nb; ++bc)
                if (bo[br * nb + bc + 1] > bo[br * nb + bc]) {
                    lo = std::min(lo, bc);
                    hi = bc + 1;
                }
            if (hi <= lo) lo = hi = 0;
            DenseRow r;
            r.lo = lo;
            r.hi = hi;
            r.off = (int32_t)off;
            r.pad = 0;
            rows.push_back(r);
            if (hi > lo) {
                DenseJob j;
                j.entry_base = dd.entry_base;
                j.blkoff_base = dd.blkoff_base;
                j.dense_base = total;
                j.nb = nb;
                j.br = br;
                j.lo = lo;
                j.hi = hi;
                j.off = (int32_t)off;
                j.pad = 0;
                jobs.push_back(j);
            }
            off += (int64_t)(hi - lo) * BB;
        }
        if (off >= INT32_MAX) return fail(CGH_EINVAL, "plane %d: dense table too large", d);
        total += off;
    }
    const size_t vb = value_bytes(lut->prm.value_dtype);
    lut->dense_zero = total;
    total += kDenseZero;
    hipError_t e1 = hipMalloc(&lut->dense_values, vb * (size_t)total);
    hipError_t e2 = hipMalloc((void **)&lut->dense_rows, sizeof(DenseRow) * rows.size());
    if (e1 != hipSuccess || e2 != hipSuccess) {
        (void)hipGetLastError();
        return fail(CGH_ENOMEM, "dense LUT allocation of %lld coefficients failed", (long long)total);
    }
    lut->device_bytes += vb * (size_t)total + sizeof(DenseRow) * rows.size();
    CGH_TRY_HIP(hipMemset(lut->dense_values, 0, vb * (size_t)total));
    CGH_TRY_HIP(hipMemcpy(lut->dense_rows, rows.data(), sizeof(DenseRow) * rows.size(), hipMemcpyHostToDevice));
    if (!jobs.empty()) {
        DenseJob *jd = nullptr;
        CGH_TRY_HIP(hipMalloc((void **)&jd, sizeof(DenseJob) * jobs.size()));
        hipError_t e = hipMemcpy(jd, jobs.data(), sizeof(DenseJob) * jobs.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(dense_scatter_kernel, dim3((unsigned)jobs.size()), dim3(256), 0, 0, jd,
                               lut->L, (int)vb, lut->blk_off, lut->keys, lut->values, lut->dense_values);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipDeviceSynchronize();
        (void)hipFree(jd);
        if (e != hipSuccess) return fail(CGH_EHIP, "dense LUT: %s", hipGetErrorString(e));
    }
    return CGH_OK;
}

// Fill the occupied block ranges, the per-plane value bound and the device descriptors.
int finish_lut(wasabi_lut *lut, const std::vector<int32_t> &blk_off_host)
{
    const int n = lut->n_tables;
    lut->max_span_px = 0;
    std::vector<float> cmax(n, 0.0f);
    {
        int64_t *eo = nullptr;
        float *cm = nullptr;
        hipError_t e = hipMalloc((void **)&eo, sizeof(int64_t) * (n + 1));
        if (e == hipSuccess) e = hipMalloc((void **)&cm, sizeof(float) * n);
        if (e == hipSuccess)
            e = hipMemcpy(eo, lut->entry_off.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            const int vt = lut->prm.value_dtype;
            if (vt == CGH_F32) hipLaunchKernelGGL(plane_cmax_kernel<CGH_F32>, dim3(n), dim3(256), 0, 0, lut->values, eo, cm);
            else if (vt == CGH_F16) hipLaunchKernelGGL(plane_cmax_kernel<CGH_F16>, dim3(n), dim3(256), 0, 0, lut->values, eo, cm);
            else hipLaunchKernelGGL(plane_cmax_kernel<CGH_BF16>, dim3(n), dim3(256), 0, 0, lut->values, eo, cm);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpy(cmax.data(), cm, sizeof(float) * n, hipMemcpyDeviceToHost);
        (void)hipFree(eo);
        (void)hipFree(cm);
        if (e != hipSuccess) return fail(CGH_EHIP, "plane bound: %s", hipGetErrorString(e));
    }
    for (int d = 0; d < n; ++d) {
        DepthDesc &dd = lut->desc_host[d];
        const int nb = dd.nb;
        const int32_t *bo = blk_off_host.data() + dd.blkoff_base;
        int br0 = nb, br1 = 0, bc0 = nb, bc1 = 0;
        for (int br = 0; br < nb; ++br)
            for (int bc = 0; bc < nb; ++bc) {
                const int b = br * nb + bc;
                if (bo[b + 1] > bo[b]) {
                    br0 = std::min(br0, br);
                    br1 = std::max(br1, br + 1);
                    bc0 = std::min(bc0, bc);
                    bc1 = std::max(bc1, bc + 1);
                }
            }
        if (br1 <= br0) br0 = br1 = bc0 = bc1 = 0;
        dd.br0 = br0;
        dd.br1 = br1;
        dd.bc0 = bc0;
        dd.bc1 = bc1;
        dd.cmax = cmax[d];
        dd.pad = 0;
        if ((int64_t)bo[(int64_t)nb * nb] != lut->Nr[d])
            return fail(CGH_EHIP, "plane %d: selected %d entries, expected %lld", d,
                        bo[(int64_t)nb * nb], (long long)lut->Nr[d]);
        lut->max_span_px = std::max(lut->max_span_px, std::max(br1 - br0, bc1 - bc0) * lut->B);
    }
    int rc = build_dense(lut, blk_off_host);
    if (rc) return rc;
    CGH_TRY_HIP(hipMemcpy(lut->desc, lut->desc_host.data(), sizeof(DepthDesc) * n, hipMemcpyHostToDevice));
    if (!lut->dense) {
        // the sparse superposition's tile buffer: 64 >> L blocks of block_stride(L) words per block row,
        // plus the row pad
        const int L = lut->L, row_words = (64 >> L) * block_stride(L) + row_pad(L);
        const int32_t wmax = *std::max_element(lut->W.begin(), lut->W.end());
        if ((int64_t)(wmax / lut->B) * row_words * 8 >= INT32_MAX)
            return fail(CGH_EINVAL, "table too large for the sparse layout's offsets");
        const size_t wb = sizeof(int32_t) * (size_t)std::max<int64_t>(lut->total_entries, 1);
        if (hipMalloc((void **)&lut->wkeys, wb) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CGH_ENOMEM, "sparse LUT offsets (%zu bytes)", wb);
        }
        lut->device_bytes += wb;
        hipLaunchKernelGGL(wide_key_kernel, dim3(n), dim3(256), 0, 0, lut->desc, lut->blk_off, lut->keys, row_words,
                           lut->wkeys);
        CGH_TRY_HIP(hipGetLastError());
        CGH_TRY_HIP(hipDeviceSynchronize());
    }
    return CGH_OK;
}

// Allocate the LUT object and its device arrays for the geometry already in lut->W / lut->Nr.
int alloc_lut(wasabi_lut *lut)
{
    const int n = lut->n_tables;
    lut->entry_off.assign(n + 1, 0);
    lut->desc_host.resize(n);
    int64_t blk_total = 0;
    for (int d = 0; d < n; ++d) {
        lut->entry_off[d + 1] = lut->entry_off[d] + lut->Nr[d];
        DepthDesc &dd = lut->desc_host[d];
        dd.W = lut->W[d];
        dd.nb = lut->W[d] / lut->B;
        dd.entry_base = lut->entry_off[d];
        dd.blkoff_base = blk_total;
        dd.dense_base = 0;
        dd.rows_base = 0;
        blk_total += (int64_t)dd.nb * dd.nb + 1;
    }
    lut->total_entries = lut->entry_off[n];
    if (lut->total_entries >= INT64_C(2147483647))
        return fail(CGH_EINVAL, "LUT of %lld entries exceeds 2^31 - 1", (long long)lut->total_entries);
    const size_t vb = value_bytes(lut->prm.value_dtype) * (size_t)std::max<int64_t>(lut->total_entries, 1);
    const size_t kb = sizeof(uint16_t) * (size_t)std::max<int64_t>(lut->total_entries, 1);
    const size_t bb = sizeof(int32_t) * (size_t)blk_total;
    const size_t db = sizeof(DepthDesc) * (size_t)n;
    hipError_t e1 = hipMalloc(&lut->values, vb);
    hipError_t e2 = hipMalloc((void **)&lut->keys, kb);
    hipError_t e3 = hipMalloc((void **)&lut->blk_off, bb);
    hipError_t e4 = hipMalloc((void **)&lut->desc, db);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
        (void)hipGetLastError();
        return fail(CGH_ENOMEM, "LUT allocation of %zu bytes failed", vb + kb + bb + db);
    }
    lut->device_bytes = vb + kb + bb + db;
    return CGH_OK;
}

wasabi_lut *new_lut(const wasabi_lut_params *prm)
{
    wasabi_lut *lut = new wasabi_lut();
    lut->prm = *prm;
    lut->L = prm->levels;
    lut->B = 1 << prm->levels;
    lut->P = 1;
    lut->n_tables = 0;
    lut->desc = nullptr;
    lut->blk_off = nullptr;
    lut->values = nullptr;
    lut->keys = nullptr;
    lut->wkeys = nullptr;
    lut->dense = false;
    lut->dense_zero = 0;
    lut->dense_values = nullptr;
    lut->dense_rows = nullptr;
    lut->device_bytes = 0;
    lut->total_entries = 0;
    lut->max_span_px = 0;
    (void)hipGetDevice(&lut->device);
    return lut;
}

template <int L>
void launch_psf_haar(int W, int nb, int sx, int sy, double z, double R2, double pitch, double lambda,
                     double2 *coef, uint32_t *magq, hipStream_t s)
{
    constexpr int BB = 1 << (2 * L);
    constexpr int G = BB >= 256 ? 1 : 256 / BB;
    const int64_t nblk = (int64_t)nb * nb;
    const unsigned grid = (unsigned)((nblk + G - 1) / G);
    ProfScope prof("psf_haar", s);
    hipLaunchKernelGGL(psf_haar_kernel<L>, dim3(grid), dim3(256), 0, s, W, nb, sx, sy, z, R2, pitch,
                       lambda, coef, magq);
}

}  // namespace
}  // namespace cgh

// =============================================================================================
extern "C" int wasabi_build_lut(const wasabi_lut_params *prm, wasabi_lut **out, void *stream)
{
    using namespace cgh;
    if (!out) return fail(CGH_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_params(prm);
    if (rc) return rc;
    wasabi_lut *lut = new_lut(prm);
    hipStream_t s = (hipStream_t)stream;
    rc = lut_geometry(lut);
    if (!rc) rc = alloc_lut(lut);
    if (rc) {
        wasabi_lut_free(lut);
        return rc;
    }
    const int n = lut->n_tables, L = lut->L;
    int64_t coef_total = 0;
    std::vector<int64_t> coef_off(n + 1, 0);
    for (int d = 0; d < n; ++d) coef_off[d + 1] = coef_off[d] + (int64_t)lut->W[d] * lut->W[d];
    coef_total = coef_off[n];
    double2 *coef = nullptr;
    uint32_t *mag2 = nullptr;
    {
        hipError_t e1 = hipMalloc((void **)&coef, sizeof(double2) * coef_total);
        hipError_t e2 = hipMalloc((void **)&mag2, sizeof(uint32_t) * coef_total);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(coef);
            (void)hipFree(mag2);
            wasabi_lut_free(lut);
            return fail(CGH_ENOMEM, "LUT build scratch of %lld coefficients failed", (long long)coef_total);
        }
    }
    const double lambda = prm->wavelength;
    std::vector<SelPlane> planes(n);
    // coiflet tables are transformed in a pixel-layout buffer of the largest table first
    double2 *tbuf = nullptr;
    DwtFilters filt;
    filt.taps = wavelet_filters(prm->wavelet, filt.lo, filt.hi);
    if (prm->wavelet != CGH_HAAR) {
        int64_t wmax = 0;
        for (int d = 0; d < n; ++d) wmax = std::max<int64_t>(wmax, lut->W[d]);
        if (hipMalloc((void **)&tbuf, sizeof(double2) * wmax * wmax) != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(CGH_ENOMEM, "coiflet table buffer of %lld coefficients failed", (long long)(wmax * wmax));
        }
    }
    for (int d = 0; d < n && !rc; ++d) {
        const int W = lut->W[d], nb = W / lut->B;
        const int ph = d % lut->P, sx = ph % lut->B, sy = ph / lut->B;  // table shift (phase tables)
        const double R2 = lut->R[d] * lut->R[d];
        double2 *c = coef + coef_off[d];
        uint32_t *m2 = mag2 + coef_off[d];
        if (prm->wavelet != CGH_HAAR) {
            ProfScope prof("psf_dwt", s);
            const int64_t cnt = (int64_t)W * W;
            const unsigned g = (unsigned)((cnt + 255) / 256);
            hipLaunchKernelGGL(psf_fill_kernel, dim3(g), dim3(256), 0, s, W, sx, sy, lut->z[d], R2, prm->pitch,
                               lambda, tbuf);
            for (int l = 0; l < L; ++l) {
                const int h = W >> l, w = W >> l;
                hipLaunchKernelGGL(dwt_line_kernel<true>, dim3(h), dim3(256), sizeof(double2) * w, s, tbuf, W, h, w, filt);
                hipLaunchKernelGGL(dwt_line_kernel<false>, dim3(w), dim3(256), sizeof(double2) * h, s, tbuf, W, h, w, filt);
            }
            hipLaunchKernelGGL(mallat_to_blocks_kernel, dim3(g), dim3(256), 0, s, tbuf, W, L, c, m2);
        } else
        switch (L) {
        case 1: launch_psf_haar<1>(W, nb, sx, sy, lut->z[d], R2, prm->pitch, lambda, c, m2, s); break;
        case 2: launch_psf_haar<2>(W, nb, sx, sy, lut->z[d], R2, prm->pitch, lambda, c, m2, s); break;
        case 3: launch_psf_haar<3>(W, nb, sx, sy, lut->z[d], R2, prm->pitch, lambda, c, m2, s); break;
        case 4: launch_psf_haar<4>(W, nb, sx, sy, lut->z[d], R2, prm->pitch, lambda, c, m2, s); break;
        case 5: launch_psf_haar<5>(W, nb, sx, sy, lut->z[d], R2, prm->pitch, lambda, c, m2, s); break;
        default: launch_psf_haar<6>(W, nb, sx, sy, lut->z[d], R2, prm->pitch, lambda, c, m2, s); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) rc = fail(CGH_EHIP, "psf_haar_kernel: %s", hipGetErrorString(e));
        const DepthDesc &dd = lut->desc_host[d];
        planes[d].coef_off = coef_off[d];
        planes[d].count = (int64_t)W * W;
        planes[d].nr = lut->Nr[d];
        planes[d].entry_base = dd.entry_base;
        planes[d].blkoff_base = dd.blkoff_base;
        planes[d].nb = nb;
        planes[d].pad = 0;
    }
    SelPlane *planes_dev = nullptr;
    if (!rc) {
        hipError_t e = hipMalloc((void **)&planes_dev, sizeof(SelPlane) * n);
        if (e == hipSuccess)
            e = hipMemcpy(planes_dev, planes.data(), sizeof(SelPlane) * n, hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = fail(CGH_EHIP, "plane table upload: %s", hipGetErrorString(e));
    }
    if (!rc) {
        ProfScope prof("select", s);
        if (prm->value_dtype == CGH_F32)
            hipLaunchKernelGGL(select_kernel<CGH_F32>, dim3(n), dim3(1024), 0, s, coef, mag2, planes_dev, L, lut->values, lut->keys, lut->blk_off);
        else if (prm->value_dtype == CGH_F16)
            hipLaunchKernelGGL(select_kernel<CGH_F16>, dim3(n), dim3(1024), 0, s, coef, mag2, planes_dev, L, lut->values, lut->keys, lut->blk_off);
        else
            hipLaunchKernelGGL(select_kernel<CGH_BF16>, dim3(n), dim3(1024), 0, s, coef, mag2, planes_dev, L, lut->values, lut->keys, lut->blk_off);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) rc = fail(CGH_EHIP, "select_kernel: %s", hipGetErrorString(e));
    }
    if (!rc) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = fail(CGH_EHIP, "LUT build: %s", hipGetErrorString(e));
    }
    (void)hipFree(coef);
    (void)hipFree(mag2);
    (void)hipFree(planes_dev);
    (void)hipFree(tbuf);
    if (!rc) {
        int64_t blk_total = lut->desc_host[n - 1].blkoff_base + (int64_t)lut->desc_host[n - 1].nb * lut->desc_host[n - 1].nb + 1;
        std::vector<int32_t> bo(blk_total);
        hipError_t e = hipMemcpy(bo.data(), lut->blk_off, sizeof(int32_t) * blk_total, hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = fail(CGH_EHIP, "hipMemcpy: %s", hipGetErrorString(e));
        if (!rc) rc = finish_lut(lut, bo);
    }
    if (rc) {
        wasabi_lut_free(lut);
        return rc;
    }
    *out = lut;
    return CGH_OK;
}

extern "C" int wasabi_lut_import(const wasabi_lut_params *prm, const int64_t *off,
                                 const int32_t *idx, const double *val, wasabi_lut **out)
{
    using namespace cgh;
    if (!out) return fail(CGH_EINVAL, "out is NULL");
    *out = nullptr;
    if (!prm) return fail(CGH_EINVAL, "params is NULL");
    wasabi_lut_params p = *prm;
    p.gamma = 1.0;  // the plane geometry does not depend on gamma; counts come from `off`
    int rc = validate_params(&p);
    if (rc) return rc;
    if (!off || !idx || !val) return fail(CGH_EINVAL, "NULL host array");
    wasabi_lut *lut = new_lut(&p);
    rc = lut_geometry(lut);
    lut->prm.gamma = prm->gamma;
    const int n = lut->n_tables, L = lut->L, B = lut->B;
    if (!rc && off[0] != 0) rc = fail(CGH_EINVAL, "off[0] must be 0");
    for (int d = 0; d < n && !rc; ++d) {
        const int64_t cnt = off[d + 1] - off[d];
        if (cnt < 0 || cnt > (int64_t)lut->W[d] * lut->W[d])
            rc = fail(CGH_EINVAL, "plane %d: bad entry count", d);
        else
            lut->Nr[d] = cnt;
    }
    if (!rc) rc = alloc_lut(lut);
    if (rc) {
        wasabi_lut_free(lut);
        return rc;
    }
    const int64_t total = lut->total_entries;
    const int BS = block_stride(L), BB = B * B;
    const int vt = prm->value_dtype;
    std::vector<uint16_t> keys(total);
    std::vector<uint32_t> packed(vt == CGH_F32 ? 2 * total : total);
    int64_t blk_total = 0;
    for (int d = 0; d < n; ++d) blk_total += (int64_t)lut->desc_host[d].nb * lut->desc_host[d].nb + 1;
    std::vector<int32_t> bo(blk_total, 0);
    for (int d = 0; d < n && !rc; ++d) {
        const int W = lut->W[d], nb = W / B;
        const int64_t o0 = off[d], cnt = off[d + 1] - off[d];
        // (sort key, canonical entry) in the internal (block row, block column, code) order
        std::vector<std::pair<int64_t, int64_t>> order(cnt);
        for (int64_t k = 0; k < cnt && !rc; ++k) {
            const int64_t f = idx[o0 + k];
            if (f < 0 || f >= (int64_t)W * W || (k > 0 && idx[o0 + k] <= idx[o0 + k - 1])) {
                rc = fail(CGH_EINVAL, "plane %d: indices must be ascending and < W^2", d);
                break;
            }
            int br, bc, code;
            flat_to_block(f, W, L, br, bc, code);
            order[k] = std::make_pair(((int64_t)br * nb + bc) * BB + code, o0 + k);
        }
        if (rc) break;
        std::sort(order.begin(), order.end());
        int32_t *bod = bo.data() + lut->desc_host[d].blkoff_base;
        int64_t pos = 0;
        for (int64_t b = 0; b <= (int64_t)nb * nb; ++b) {
            while (pos < cnt && order[pos].first / BB < b) ++pos;
            bod[b] = (int32_t)pos;
        }
        for (int64_t k = 0; k < cnt; ++k) {
            const int64_t sk = order[k].first, src = order[k].second;
            const int64_t blk = sk / BB;
            const int code = (int)(sk % BB);
            const int64_t at = o0 + k;
            keys[at] = (uint16_t)((blk % nb) * BS + code);
            const double re = val[2 * src], im = val[2 * src + 1];
            if (vt == CGH_F32) {
                const float fr = (float)re, fi = (float)im;
                memcpy(&packed[2 * at], &fr, 4);
                memcpy(&packed[2 * at + 1], &fi, 4);
            } else if (vt == CGH_F16) {
                packed[at] = f64_to_f16_bits(re) | (f64_to_f16_bits(im) << 16);
            } else {
                packed[at] = f64_to_bf16_bits(re) | (f64_to_bf16_bits(im) << 16);
            }
        }
    }
    if (!rc && total > 0) {
        hipError_t e1 = hipMemcpy(lut->keys, keys.data(), sizeof(uint16_t) * total, hipMemcpyHostToDevice);
        hipError_t e2 = hipMemcpy(lut->values, packed.data(), sizeof(uint32_t) * packed.size(), hipMemcpyHostToDevice);
        if (e1 != hipSuccess || e2 != hipSuccess) rc = fail(CGH_EHIP, "LUT upload failed");
    }
    if (!rc) {
        hipError_t e = hipMemcpy(lut->blk_off, bo.data(), sizeof(int32_t) * blk_total, hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = fail(CGH_EHIP, "LUT upload failed");
    }
    if (!rc) rc = finish_lut(lut, bo);
    if (rc) {
        wasabi_lut_free(lut);
        return rc;
    }
    *out = lut;
    return CGH_OK;
}

extern "C" int wasabi_lut_info(const wasabi_lut *lut, int32_t *n_tables, int64_t *total_entries,
                               int64_t *device_bytes, double *z, double *R, int32_t *W, int64_t *Nr)
{
    using namespace cgh;
    if (!lut) return fail(CGH_EINVAL, "lut is NULL");
    const int n = lut->n_tables;
    if (n_tables) *n_tables = n;
    if (total_entries) *total_entries = lut->total_entries;
    if (device_bytes) *device_bytes = (int64_t)lut->device_bytes;
    for (int d = 0; d < n; ++d) {
        if (z) z[d] = lut->z[d];
        if (R) R[d] = lut->R[d];
        if (W) W[d] = lut->W[d];
        if (Nr) Nr[d] = lut->Nr[d];
    }
    return CGH_OK;
}

extern "C" int wasabi_lut_export(const wasabi_lut *lut, int64_t *off, int32_t *idx, double *val)
{
    using namespace cgh;
    if (!lut || !off || !idx || !val) return fail(CGH_EINVAL, "NULL argument");
    const int n = lut->n_tables, L = lut->L, B = lut->B, BS = block_stride(L);
    const int64_t total = lut->total_entries;
    const int vt = lut->prm.value_dtype;
    std::vector<uint16_t> keys(total);
    std::vector<uint32_t> packed(vt == CGH_F32 ? 2 * total : total);
    int64_t blk_total = 0;
    for (int d = 0; d < n; ++d) blk_total += (int64_t)lut->desc_host[d].nb * lut->desc_host[d].nb + 1;
    std::vector<int32_t> bo(blk_total);
    if (total > 0) {
        CGH_TRY_HIP(hipMemcpy(keys.data(), lut->keys, sizeof(uint16_t) * total, hipMemcpyDeviceToHost));
        CGH_TRY_HIP(hipMemcpy(packed.data(), lut->values, sizeof(uint32_t) * packed.size(), hipMemcpyDeviceToHost));
    }
    CGH_TRY_HIP(hipMemcpy(bo.data(), lut->blk_off, sizeof(int32_t) * blk_total, hipMemcpyDeviceToHost));
    for (int d = 0; d <= n; ++d) off[d] = lut->entry_off[d];
    for (int d = 0; d < n; ++d) {
        const DepthDesc &dd = lut->desc_host[d];
        const int nb = dd.nb;
        const int32_t *bod = bo.data() + dd.blkoff_base;
        std::vector<std::pair<int64_t, int64_t>> order;
        order.reserve(lut->Nr[d]);
        for (int br = 0; br < nb; ++br) {
            for (int bc = 0; bc < nb; ++bc) {
                const int b = br * nb + bc;
                for (int32_t k = bod[b]; k < bod[b + 1]; ++k) {
                    const int64_t at = dd.entry_base + k;
                    const int code = keys[at] - (keys[at] / BS) * BS;
                    order.emplace_back(block_to_flat(br, bc, code, dd.W, L), at);
                }
            }
        }
        std::sort(order.begin(), order.end());
        for (size_t k = 0; k < order.size(); ++k) {
            const int64_t o = dd.entry_base + (int64_t)k, at = order[k].second;
            idx[o] = (int32_t)order[k].first;
            if (vt == CGH_F32) {
                float fr, fi;
                memcpy(&fr, &packed[2 * at], 4);
                memcpy(&fi, &packed[2 * at + 1], 4);
                val[2 * o] = fr;
                val[2 * o + 1] = fi;
            } else if (vt == CGH_F16) {
                val[2 * o] = f16_bits_to_f64(packed[at] & 0xffff);
                val[2 * o + 1] = f16_bits_to_f64(packed[at] >> 16);
            } else {
                val[2 * o] = bf16_bits_to_f64(packed[at] & 0xffff);
                val[2 * o + 1] = bf16_bits_to_f64(packed[at] >> 16);
            }
        }
        (void)B;
    }
    return CGH_OK;
}

extern "C" void wasabi_lut_free(wasabi_lut *lut)
{
    if (!lut) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(lut->desc);
    (void)hipFree(lut->blk_off);
    (void)hipFree(lut->values);
    (void)hipFree(lut->keys);
    (void)hipFree(lut->wkeys);
    (void)hipFree(lut->dense_values);
    (void)hipFree(lut->dense_rows);
    delete lut;
}

namespace cgh {
int quantize_shifted(const wasabi_lut *lut, const double *pts, int64_t n, double z_shift,
                     wasabi_point *out, hipStream_t stream)
{
    if (!lut) return fail(CGH_EINVAL, "lut is NULL");
    if (n < 0) return fail(CGH_EINVAL, "n < 0");
    if (n == 0) return CGH_OK;
    if (!pts || !out) return fail(CGH_EINVAL, "NULL pointer");
    const wasabi_lut_params &p = lut->prm;
    const double dz = (p.z_max - p.z_min) / (double)p.n_depth;
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    if (blocks > INT32_MAX) return fail(CGH_EINVAL, "n too large");
    ProfScope prof("quantize", (hipStream_t)stream);
    hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)blocks), dim3(threads), 0, (hipStream_t)stream,
                       (const double4 *)pts, n, p.pitch, p.z_min, p.z_max, dz, p.n_depth, lut->L,
                       p.phases, z_shift, out);
    CGH_CHECK_LAUNCH("quantize_kernel");
    return CGH_OK;
}
}  // namespace cgh

extern "C" int wasabi_quantize(const wasabi_lut *lut, const double *pts, int64_t n,
                               wasabi_point *out, void *stream)
{
    return cgh::quantize_shifted(lut, pts, n, 0.0, out, (hipStream_t)stream);
}
