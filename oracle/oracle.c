/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the WASABI hologram path
 * (Shimobaba et al., "Fast, large-scale hologram calculation in wavelet domain").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg do.  It shares
 * no code, header or constant generator with the HIP path.
 *
 * Every routine follows one passage of the paper, written as loops that can be checked by eye:
 *   oracle_direct        Eq.(1): u(x_h,y_h) = sum_j a_j exp(i 2 pi r_hj / lambda), with an
 *                        optional circ() window (the PSF support of Sec. 2, step 1).
 *   oracle_lut_geometry  Sec. 2, step 1: depth planes spaced by dz, PSF radius, N_r = gamma*pi*R^2.
 *   oracle_psf_table     Sec. 2, step 1: u_z = exp(i k r) circ(.) sampled on a W x W table.
 *   oracle_haar_forward  Sec. 2, step 1 / Fig. 2(a): L-level fast wavelet transform (Haar,
 *   oracle_haar_inverse  orthonormal, Mallat layout) and its inverse (Sec. 2, step 3).
 *   oracle_dwt_forward   the same with coiflets, the wavelet the paper names (Sec. 2): periodised
 *   oracle_dwt_inverse   separable filter banks; Haar's filters give the Haar transform.
 *   oracle_select        Sec. 2, step 1: keep the N_r strongest coefficients.
 *   oracle_quantize      depth discretisation (Sec. 2, step 1) and the 2^L position grid that
 *                        makes the level-scaled shift of Eq.(2) an integer; with phase tables,
 *                        the pixel grid and the point's position inside its 2^L block.
 *   oracle_superpose     Eq.(2) with the sub-hologram coordinate shift x'_j = x_j - s N_h
 *                        (Sec. 2, large-scale procedure, steps 2-3).
 *
 * Readings of passages the paper leaves open (window radius, tie-breaking, sub-band layout,
 * plane centres ...) are the ones listed in the design notes; each is restated where used.
 * Complex arrays are interleaved (re, im) doubles, row-major, row = y, column = x.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* sin(theta_max) = lambda / (2 p): the largest diffraction angle a pitch-p grid can record. */
static double tan_theta_max(double wavelength, double pitch)
{
    double s = wavelength / (2.0 * pitch);
    return s / sqrt(1.0 - s * s);
}

/* ------------------------------------------------------------------------------------------
 * Eq.(1).  pts: n x {x, y, z, a} in metres (x, y relative to the centre of global pixel (0,0)).
 * Output pixel (i, j) of the ny x nx window sits at ((ox + j) p, (oy + i) p).
 * window = 0: every point reaches every pixel (Eq.(1) literally).
 * window = 1: a point reaches a pixel only inside its PSF disk, rho^2 < (z tan theta_max)^2,
 *             i.e. the circ() support of the pre-computed PSF (Sec. 2, step 1).
 * out: ny x nx complex (interleaved doubles).
 * ---------------------------------------------------------------------------------------- */
void oracle_direct(const double *pts, int64_t n, int32_t nx, int32_t ny, int64_t ox, int64_t oy,
                   double pitch, double wavelength, int32_t window, double *out)
{
    const double tan_t = tan_theta_max(wavelength, pitch);
    int32_t i;
#pragma omp parallel for schedule(dynamic, 1)
    for (i = 0; i < ny; i++) {
        for (int32_t j = 0; j < nx; j++) {
            const double xh = (double)(ox + j) * pitch;
            const double yh = (double)(oy + i) * pitch;
            double re = 0.0, im = 0.0;
            for (int64_t k = 0; k < n; k++) {
                const double x = pts[4 * k + 0], y = pts[4 * k + 1];
                const double z = pts[4 * k + 2], a = pts[4 * k + 3];
                const double dx = xh - x, dy = yh - y;
                const double rho2 = dx * dx + dy * dy;
                if (window) {
                    const double R = z * tan_t;
                    if (!(rho2 < R * R)) continue;
                }
                const double r = sqrt(rho2 + z * z);
                const double phase = 2.0 * M_PI * r / wavelength;
                re += a * cos(phase);
                im += a * sin(phase);
            }
            out[2 * ((int64_t)i * nx + j) + 0] = re;
            out[2 * ((int64_t)i * nx + j) + 1] = im;
        }
    }
}

/* ------------------------------------------------------------------------------------------
 * Plane geometry (Sec. 2, step 1; Sec. 3 uses dz = depth range / N_z).
 *   dz  = (z_max - z_min) / n_depth,  plane d sits at the cell centre z_d = z_min + (d + 1/2) dz
 *   R_d = z_d tan(theta_max) / p     PSF radius in pixels (the circ() support)
 *   W_d = table side: the smallest multiple of 2^(L+1) that holds the disk, W_d >= 2 floor(R_d) + 2,
 *         so that the table centre W_d / 2 is a multiple of 2^L.  With phase tables the disk's
 *         centre may sit up to 2^L - 1 pixels right of / below the table centre, so the table
 *         must hold a disk around any of those centres: W_d >= 2 floor(R_d) + 2^(L+1).  Coiflet
 *         tables add a margin of 5 2^L pixels on each side.
 *   N_r = ceil(gamma pi R_d^2) clamped to [1, W_d^2]; gamma >= 1 keeps all W_d^2 coefficients.
 * Returns 0, or -1 if a table would exceed max_window.
 * ---------------------------------------------------------------------------------------- */
int oracle_lut_geometry(double wavelength, double pitch, double z_min, double z_max, int32_t n_depth,
                        int32_t levels, int32_t max_window, double gamma, int32_t phases,
                        int32_t wavelet, double *z, double *R, int32_t *W, int64_t *Nr)
{
    const double tan_t = tan_theta_max(wavelength, pitch);
    const double dz = (z_max - z_min) / (double)n_depth;
    const int32_t q = 1 << (levels + 1);
    for (int32_t d = 0; d < n_depth; d++) {
        z[d] = z_min + ((double)d + 0.5) * dz;
        R[d] = z[d] * tan_t / pitch;
        int32_t need = 2 * (int32_t)floor(R[d]) + (phases ? q : 2);
        /* coiflet tables: the periodised transform moves a coefficient up to 5 (2^L - 1) pixels
           from its support, so a margin of 5 2^L on each side keeps the disk's coefficients from
           wrapping round the table */
        if (wavelet == 1) need += 2 * 5 * (1 << levels);
        W[d] = ((need + q - 1) / q) * q;
        if (W[d] > max_window) return -1;
        int64_t all = (int64_t)W[d] * W[d];
        if (gamma >= 1.0) {
            Nr[d] = all;
        } else {
            double want = ceil(gamma * M_PI * R[d] * R[d]);
            int64_t k = (int64_t)want;
            if (k < 1) k = 1;
            if (k > all) k = all;
            Nr[d] = k;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * PSF table (Sec. 2, step 1):  T[r][q] = exp(i 2 pi / lambda * sqrt(((q-cx)p)^2 + ((r-cy)p)^2 + z^2))
 * when (q-cx)^2 + (r-cy)^2 < R^2 (circ(c) = 1 iff c < 1), else 0.  The disk's centre is
 * (cx, cy) = (W/2 + sx, W/2 + sy): sx = sy = 0 for the paper's one table per plane; a phase table
 * holds the PSF of a point sx columns right of and sy rows below its 2^L block's corner.
 * The phase is taken modulo one revolution before the cosine and sine: the same value, but the
 * thousands of whole revolutions no longer cost FP64 digits.
 * ---------------------------------------------------------------------------------------- */
void oracle_psf_table(double z, double R, int32_t W, int32_t sx, int32_t sy, double pitch,
                      double wavelength, double *T)
{
    const int32_t cx = W / 2 + sx, cy = W / 2 + sy;
    for (int32_t r = 0; r < W; r++) {
        for (int32_t q = 0; q < W; q++) {
            const double dq = (double)(q - cx), dr = (double)(r - cy);
            double re = 0.0, im = 0.0;
            if (dq * dq + dr * dr < R * R) {
                /* phase 2 pi dist / lambda, whole revolutions removed first (an exact step) */
                const double dist = sqrt((dq * pitch) * (dq * pitch) + (dr * pitch) * (dr * pitch) + z * z);
                const double rev = dist / wavelength;
                const double frac = rev - floor(rev);
                re = cos(2.0 * M_PI * frac);
                im = sin(2.0 * M_PI * frac);
            }
            T[2 * ((int64_t)r * W + q) + 0] = re;
            T[2 * ((int64_t)r * W + q) + 1] = im;
        }
    }
}

/* ------------------------------------------------------------------------------------------
 * Orthonormal 2D Haar, one level on the top-left h x w region of an array with row stride
 * `stride` (complex elements).  For the 2x2 block a=A[2m][2n], b=A[2m][2n+1], c=A[2m+1][2n],
 * d=A[2m+1][2n+1]:
 *     S = (a+b+c+d)/2 -> top-left quadrant      H = (a-b+c-d)/2 -> top-right
 *     V = (a+b-c-d)/2 -> bottom-left            D = (a-b-c+d)/2 -> bottom-right
 * The scaling quadrant S is transformed again at the next level (Fig. 2(a) layout).
 * ---------------------------------------------------------------------------------------- */
static void haar_forward_level(double *A, int32_t h, int32_t w, int64_t stride)
{
    const int32_t h2 = h / 2, w2 = w / 2;
    double *t = (double *)malloc(sizeof(double) * 2 * (size_t)h * (size_t)w);
    for (int32_t m = 0; m < h2; m++) {
        for (int32_t n = 0; n < w2; n++) {
            for (int ri = 0; ri < 2; ri++) {
                const double a = A[2 * ((int64_t)(2 * m) * stride + 2 * n) + ri];
                const double b = A[2 * ((int64_t)(2 * m) * stride + 2 * n + 1) + ri];
                const double c = A[2 * ((int64_t)(2 * m + 1) * stride + 2 * n) + ri];
                const double d = A[2 * ((int64_t)(2 * m + 1) * stride + 2 * n + 1) + ri];
                t[2 * ((int64_t)m * w + n) + ri] = (a + b + c + d) / 2.0;
                t[2 * ((int64_t)m * w + w2 + n) + ri] = (a - b + c - d) / 2.0;
                t[2 * ((int64_t)(h2 + m) * w + n) + ri] = (a + b - c - d) / 2.0;
                t[2 * ((int64_t)(h2 + m) * w + w2 + n) + ri] = (a - b - c + d) / 2.0;
            }
        }
    }
    for (int32_t r = 0; r < h; r++)
        memcpy(&A[2 * (int64_t)r * stride], &t[2 * (int64_t)r * w], sizeof(double) * 2 * (size_t)w);
    free(t);
}

/* Inverse of haar_forward_level:  a = (S+H+V+D)/2, b = (S-H+V-D)/2, c = (S+H-V-D)/2, d = (S-H-V+D)/2. */
static void haar_inverse_level(double *A, int32_t h, int32_t w, int64_t stride)
{
    const int32_t h2 = h / 2, w2 = w / 2;
    double *t = (double *)malloc(sizeof(double) * 2 * (size_t)h * (size_t)w);
    for (int32_t m = 0; m < h2; m++) {
        for (int32_t n = 0; n < w2; n++) {
            for (int ri = 0; ri < 2; ri++) {
                const double S = A[2 * ((int64_t)m * stride + n) + ri];
                const double H = A[2 * ((int64_t)m * stride + w2 + n) + ri];
                const double V = A[2 * ((int64_t)(h2 + m) * stride + n) + ri];
                const double D = A[2 * ((int64_t)(h2 + m) * stride + w2 + n) + ri];
                t[2 * ((int64_t)(2 * m) * w + 2 * n) + ri] = (S + H + V + D) / 2.0;
                t[2 * ((int64_t)(2 * m) * w + 2 * n + 1) + ri] = (S - H + V - D) / 2.0;
                t[2 * ((int64_t)(2 * m + 1) * w + 2 * n) + ri] = (S + H - V - D) / 2.0;
                t[2 * ((int64_t)(2 * m + 1) * w + 2 * n + 1) + ri] = (S - H - V + D) / 2.0;
            }
        }
    }
    for (int32_t r = 0; r < h; r++)
        memcpy(&A[2 * (int64_t)r * stride], &t[2 * (int64_t)r * w], sizeof(double) * 2 * (size_t)w);
    free(t);
}

/* L-level transform of an h x w complex array in place (h, w multiples of 2^L). */
void oracle_haar_forward(double *A, int32_t h, int32_t w, int32_t levels)
{
    for (int32_t l = 0; l < levels; l++) haar_forward_level(A, h >> l, w >> l, w);
}

void oracle_haar_inverse(double *A, int32_t h, int32_t w, int32_t levels)
{
    for (int32_t l = levels - 1; l >= 0; l--) haar_inverse_level(A, h >> l, w >> l, w);
}

/* ------------------------------------------------------------------------------------------
 * Filter banks.  wavelet 0: Haar, lo = (1, 1)/sqrt 2.  wavelet 1: the coiflet of order 1 (six
 * taps).  The paper uses coiflets at level 3 without naming the order; the shortest is taken.
 * Its scaling filter has the closed form (Daubechies, Ten Lectures on Wavelets, Sec. 8.2)
 *     lo = sqrt(2)/32 (1 - s, 5 + s, 14 + 2s, 14 - 2s, 1 - s, -3 + s),   s = sqrt 7,
 * and the wavelet filter is hi[n] = (-1)^n lo[taps - 1 - n].  Returns the number of taps.
 * ---------------------------------------------------------------------------------------- */
int32_t oracle_filters(int32_t wavelet, double *lo, double *hi)
{
    int32_t taps;
    if (wavelet == 1) {
        const double s = sqrt(7.0), c = sqrt(2.0) / 32.0;
        const double f[6] = {1 - s, 5 + s, 14 + 2 * s, 14 - 2 * s, 1 - s, -3 + s};
        taps = 6;
        for (int32_t n = 0; n < taps; n++) lo[n] = c * f[n];
    } else {
        taps = 2;
        lo[0] = lo[1] = 1.0 / sqrt(2.0);
    }
    for (int32_t n = 0; n < taps; n++) hi[n] = ((n & 1) ? -1.0 : 1.0) * lo[taps - 1 - n];
    return taps;
}

/* One level of the periodised orthonormal 2-D transform of the top-left h x w region of an
 * array with row stride `stride` (complex elements).  Along every row of length w:
 *     a[k] = sum_t lo[t] x[(2k + t) mod w],   d[k] = sum_t hi[t] x[(2k + t) mod w],
 * a into the left half, d into the right half; then the same along every column (a on top, d
 * below).  So the quadrants are S (top-left, transformed again at the next level), H = detail
 * along x (top-right), V = detail along y (bottom-left), D (bottom-right), as for Haar. */
static void dwt_1d(const double *x, double *out, int32_t len, int64_t step, const double *lo,
                   const double *hi, int32_t taps, int inverse)
{
    /* x and out: len complex values, `step` complex elements apart */
    const int32_t half = len / 2;
    double *t = (double *)calloc(2 * (size_t)len, sizeof(double));
    for (int32_t k = 0; k < half; k++) {
        for (int32_t j = 0; j < taps; j++) {
            const int64_t n = (2 * (int64_t)k + j) % len;
            for (int ri = 0; ri < 2; ri++) {
                if (!inverse) {
                    t[2 * k + ri] += lo[j] * x[2 * n * step + ri];
                    t[2 * (half + k) + ri] += hi[j] * x[2 * n * step + ri];
                } else {   /* the transpose: x[n] += a[k] lo[j] + d[k] hi[j] */
                    t[2 * n + ri] += lo[j] * x[2 * (int64_t)k * step + ri] + hi[j] * x[2 * (int64_t)(half + k) * step + ri];
                }
            }
        }
    }
    for (int32_t i = 0; i < len; i++) {
        out[2 * (int64_t)i * step] = t[2 * i];
        out[2 * (int64_t)i * step + 1] = t[2 * i + 1];
    }
    free(t);
}

void oracle_dwt_forward(double *A, int32_t h, int32_t w, int32_t levels, int32_t wavelet)
{
    double lo[8], hi[8];
    const int32_t taps = oracle_filters(wavelet, lo, hi);
    for (int32_t l = 0; l < levels; l++) {
        const int32_t hl = h >> l, wl = w >> l;
        for (int32_t r = 0; r < hl; r++) dwt_1d(A + 2 * (int64_t)r * w, A + 2 * (int64_t)r * w, wl, 1, lo, hi, taps, 0);
        for (int32_t c = 0; c < wl; c++) dwt_1d(A + 2 * (int64_t)c, A + 2 * (int64_t)c, hl, w, lo, hi, taps, 0);
    }
}

/* Inverse of oracle_dwt_forward: per level, coarsest first, columns then rows, each the transpose
 * of the forward step (the filter bank is orthonormal). */
void oracle_dwt_inverse(double *A, int32_t h, int32_t w, int32_t levels, int32_t wavelet)
{
    double lo[8], hi[8];
    const int32_t taps = oracle_filters(wavelet, lo, hi);
    for (int32_t l = levels - 1; l >= 0; l--) {
        const int32_t hl = h >> l, wl = w >> l;
        for (int32_t c = 0; c < wl; c++) dwt_1d(A + 2 * (int64_t)c, A + 2 * (int64_t)c, hl, w, lo, hi, taps, 1);
        for (int32_t r = 0; r < hl; r++) dwt_1d(A + 2 * (int64_t)r * w, A + 2 * (int64_t)r * w, wl, 1, lo, hi, taps, 1);
    }
}

/* ------------------------------------------------------------------------------------------
 * Shrinkage (Sec. 2, step 1): keep the N_r strongest coefficients.  Strength is |c|^2 computed
 * in FP64 and rounded to single precision (24 significant bits); equal strengths go to the lower
 * flat index (idx = row * W + col).  The rounding makes coefficients that are equal in exact
 * arithmetic (e.g. the transposed twins of the symmetric PSF) compare equal, so the kept set
 * does not depend on last-bit rounding noise.  The kept entries are written sorted by flat
 * index.  C: W x W complex.
 * ---------------------------------------------------------------------------------------- */
typedef struct { float mag2; int32_t idx; } mag_entry;

static int by_magnitude_then_index(const void *pa, const void *pb)
{
    const mag_entry *a = (const mag_entry *)pa, *b = (const mag_entry *)pb;
    if (a->mag2 > b->mag2) return -1;
    if (a->mag2 < b->mag2) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

static int by_index(const void *pa, const void *pb)
{
    const int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    return (a > b) - (a < b);
}

void oracle_select(const double *C, int32_t W, int64_t Nr, int32_t *idx_out, double *val_out)
{
    const int64_t all = (int64_t)W * W;
    mag_entry *e = (mag_entry *)malloc(sizeof(mag_entry) * (size_t)all);
    for (int64_t k = 0; k < all; k++) {
        e[k].mag2 = (float)(C[2 * k] * C[2 * k] + C[2 * k + 1] * C[2 * k + 1]);
        e[k].idx = (int32_t)k;
    }
    qsort(e, (size_t)all, sizeof(mag_entry), by_magnitude_then_index);
    for (int64_t k = 0; k < Nr; k++) idx_out[k] = e[k].idx;
    qsort(idx_out, (size_t)Nr, sizeof(int32_t), by_index);
    for (int64_t k = 0; k < Nr; k++) {
        val_out[2 * k + 0] = C[2 * (int64_t)idx_out[k] + 0];
        val_out[2 * k + 1] = C[2 * (int64_t)idx_out[k] + 1];
    }
    free(e);
}

/* ------------------------------------------------------------------------------------------
 * Storage rounding of LUT values, round-to-nearest-even from FP64.
 * dtype 0 = FP32, 1 = FP16 (11 significant bits, min normal 2^-14, max 65504),
 *       2 = BF16 (8 significant bits, float32 exponent range), 3 = FP64 (kept as computed).  Written from the IEEE 754
 * definition: v = m 2^e with 0.5 <= |m| < 1; the quantum is 2^(max(e, e_min) - bits).
 * ---------------------------------------------------------------------------------------- */
static double round_to_bits(double v, int bits, int e_min, double max_finite)
{
    if (v == 0.0 || !isfinite(v)) return v;
    int e;
    (void)frexp(v, &e);
    if (e < e_min) e = e_min;
    const double quantum = ldexp(1.0, e - bits);
    const double r = nearbyint(v / quantum) * quantum; /* default rounding mode: ties to even */
    if (fabs(r) > max_finite) return copysign(INFINITY, v);
    return r;
}

double oracle_round_value(double v, int32_t dtype)
{
    if (dtype == 3) return v;
    if (dtype == 0) return (double)(float)v;
    if (dtype == 1) return round_to_bits(v, 11, -13, 65504.0);
    return round_to_bits(v, 8, -125, 3.3895313892515355e38);
}

/* ------------------------------------------------------------------------------------------
 * LUT build (Sec. 2, step 1): for every table, PSF table -> L-level wavelet transform (Haar, or
 * the coiflet with wavelet = 1) -> N_r strongest
 * coefficients -> values rounded to the storage dtype.  Canonical layout: table d owns
 * entries [off[d], off[d+1]), sorted by flat table index.  off has n_tables + 1 entries and is
 * computed by the caller from Nr (off[0] = 0).  Table d's disk centre is shifted by
 * (sx[d], sy[d]) pixels from the table centre (all zero without phase tables).
 * ---------------------------------------------------------------------------------------- */
void oracle_build_lut(double wavelength, double pitch, int32_t n_tables, int32_t levels,
                      const double *z, const double *R, const int32_t *W, const int64_t *Nr,
                      const int32_t *sx, const int32_t *sy, const int64_t *off, int32_t value_dtype,
                      int32_t wavelet, int32_t *idx, double *val)
{
    for (int32_t d = 0; d < n_tables; d++) {
        double *T = (double *)malloc(sizeof(double) * 2 * (size_t)W[d] * (size_t)W[d]);
        oracle_psf_table(z[d], R[d], W[d], sx[d], sy[d], pitch, wavelength, T);
        if (wavelet == 0)
            oracle_haar_forward(T, W[d], W[d], levels);
        else
            oracle_dwt_forward(T, W[d], W[d], levels, wavelet);
        oracle_select(T, W[d], Nr[d], idx + off[d], val + 2 * off[d]);
        for (int64_t k = 2 * off[d]; k < 2 * off[d + 1]; k++) val[k] = oracle_round_value(val[k], value_dtype);
        free(T);
    }
}

/* floor(v / 2^s) for any sign of v. */
static int64_t floor_shift(int64_t v, int32_t s)
{
    const int64_t q = (int64_t)1 << s;
    int64_t r = v / q;
    if (r * q > v) r -= 1;
    return r;
}

/* ------------------------------------------------------------------------------------------
 * Point quantisation.  x, y (metres) -> the nearest multiple of 2^L pixels (ties upward), so
 * that the level-scaled shift of Eq.(2) lands on integer coefficient positions at every level;
 * z -> plane d = floor((z - z_min) / dz), with z = z_max going to the last plane (Sec. 2,
 * step 1, depth discretisation).  Points with z outside [z_min, z_max], a non-finite
 * coordinate, or a snapped position beyond +-2^30 pixels get d = -1 and contribute nothing.
 * With phase tables (phases = 1) x, y go to the nearest pixel instead (ties upward) and the
 * table index is d 4^L + (y mod 2^L) 2^L + (x mod 2^L): the table of the point's position
 * inside its 2^L block (mod taken towards minus infinity).
 * ---------------------------------------------------------------------------------------- */
void oracle_quantize(const double *pts, int64_t n, double pitch, double z_min, double z_max,
                     int32_t n_depth, int32_t levels, int32_t phases, int32_t *qx, int32_t *qy,
                     int32_t *qd, double *qa)
{
    const double B = (double)(phases ? 1 : (1 << levels));
    const double dz = (z_max - z_min) / (double)n_depth;
    for (int64_t k = 0; k < n; k++) {
        const double x = pts[4 * k], y = pts[4 * k + 1], z = pts[4 * k + 2], a = pts[4 * k + 3];
        qa[k] = a;
        qx[k] = 0;
        qy[k] = 0;
        qd[k] = -1;
        if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !isfinite(a)) continue;
        if (z < z_min || z > z_max) continue;
        const double sx = B * floor(x / pitch / B + 0.5);
        const double sy = B * floor(y / pitch / B + 0.5);
        if (fabs(sx) >= 1073741824.0 || fabs(sy) >= 1073741824.0) continue;
        int32_t d = (int32_t)floor((z - z_min) / dz);
        if (d > n_depth - 1) d = n_depth - 1;
        qx[k] = (int32_t)sx;
        qy[k] = (int32_t)sy;
        if (phases) {
            const int64_t px = (int64_t)sx - (floor_shift((int64_t)sx, levels) << levels);
            const int64_t py = (int64_t)sy - (floor_shift((int64_t)sy, levels) << levels);
            d = (int32_t)(((int64_t)d << (2 * levels)) + (py << levels) + px);
        }
        qd[k] = d;
    }
}

/* ------------------------------------------------------------------------------------------
 * Eq.(2) on the ny x nx sub-hologram whose pixel (0,0) is global pixel (X0, Y0) (Sec. 2,
 * large-scale steps 2-3: x'_j = x_j - X0, y'_j = y_j - Y0).  psi: ny x nx complex, Mallat layout
 * (level-l bands of size (ny>>l) x (nx>>l): H at (0, nx>>l), V at (ny>>l, 0), D at (ny>>l, nx>>l);
 * S^(L) at (0,0)), accumulated in place.
 *
 * The table of point j is table d = pd[j] (its plane, or its plane and phase).
 * A kept entry at flat index idx of plane d's W x W table sits at table row/col (row, col).  Its
 * level l and band follow from the Mallat layout: the first l = 1..L with row >= W>>l or
 * col >= W>>l, else the scaling band at level L.  The table's pixel (0,0) lies at global pixel
 * (x_j - W/2, y_j - W/2); at level l that origin moves by 2^-l (the shift weight alpha of Eq.(2)),
 * so the entry lands at band position (m + floor(oy / 2^l), n + floor(ox / 2^l)) with
 * ox = x_j - W/2 - X0, oy = y_j - W/2 - Y0.  Entries landing outside the sub-hologram are dropped.
 * x_j, y_j are first floored to multiples of 2^L (the identity for points snapped to the 2^L
 * grid; for a point with a phase table, the corner of its 2^L block, the table carrying the rest).
 * ---------------------------------------------------------------------------------------- */
void oracle_superpose(int32_t levels, const int32_t *W, const int64_t *off, const int32_t *idx,
                      const double *val, const int32_t *px, const int32_t *py, const int32_t *pd,
                      const double *pa, int64_t n, int64_t X0, int64_t Y0, int32_t nx, int32_t ny,
                      double *psi)
{
    for (int64_t j = 0; j < n; j++) {
        const int32_t d = pd[j];
        if (d < 0) continue;
        const int64_t xg = floor_shift(px[j], levels) << levels;
        const int64_t yg = floor_shift(py[j], levels) << levels;
        const int64_t ox = xg - W[d] / 2 - X0;
        const int64_t oy = yg - W[d] / 2 - Y0;
        for (int64_t k = off[d]; k < off[d + 1]; k++) {
            const int32_t row = idx[k] / W[d], col = idx[k] % W[d];
            int32_t lev = levels, band = 0, m = row, nn = col;
            for (int32_t l = 1; l <= levels; l++) {
                const int32_t s = W[d] >> l;
                if (row >= s || col >= s) {
                    lev = l;
                    band = 2 * (row >= s) + (col >= s); /* 1 = H, 2 = V, 3 = D */
                    m = row - (row >= s ? s : 0);
                    nn = col - (col >= s ? s : 0);
                    break;
                }
            }
            const int64_t tm = m + floor_shift(oy, lev);
            const int64_t tn = nn + floor_shift(ox, lev);
            const int64_t bh = ny >> lev, bw = nx >> lev;
            if (tm < 0 || tm >= bh || tn < 0 || tn >= bw) continue;
            const int64_t row0 = (band == 2 || band == 3) ? bh : 0;
            const int64_t col0 = (band == 1 || band == 3) ? bw : 0;
            const int64_t at = (row0 + tm) * nx + col0 + tn;
            psi[2 * at + 0] += pa[j] * val[2 * k + 0];
            psi[2 * at + 1] += pa[j] * val[2 * k + 1];
        }
    }
}
