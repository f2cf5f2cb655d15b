/*
 * cgh.h -- C ABI of the MI355X (gfx950) WASABI hologram library, libcgh.so.
 *
 * Method: T. Shimobaba et al., "Fast, large-scale hologram calculation in wavelet domain"
 * (WAvelet ShrinkAge-Based superpositIon).  A hologram of N point sources is
 *     u(x_h, y_h) = sum_j a_j exp(i 2 pi r_hj / lambda)                          (Eq.(1))
 * WASABI computes it by superposing, in the wavelet domain, the N_r strongest wavelet
 * coefficients of each point's pre-computed PSF at level-scaled shifts (Eq.(2)), then running one
 * inverse wavelet transform (Sec. 2, steps 1-3); large holograms are split into sub-holograms
 * (Sec. 2, large-scale procedure).  The wavelet here is the orthonormal Haar wavelet.
 *
 * Conventions for every call
 *  - Pointers named *_dev / buffers documented as "device" are device memory of the current HIP
 *    device; the caller owns them and the library never frees them.  Host buffers are named as such.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Calls enqueue work on
 *    it and return without waiting, except where a call says it synchronises.
 *  - Coordinates: pixel (i, j) of a window with origin (ox, oy) is global pixel (ox + j, oy + i);
 *    row = y, column = x; the centre of global pixel (0, 0) is the physical origin.
 *  - Complex data is interleaved (re, im): complex64 = 2 x float, complex128 = 2 x double.
 *  - Every call validates its arguments before launching anything and returns CGH_OK or a negative
 *    cgh_status; cgh_last_error() then gives a message (thread-local).  A kernel launch failure is
 *    reported by the call that launched it; faults that occur later surface at the caller's next
 *    synchronisation of the stream.
 *  - Scratch memory is taken from HIP's stream-ordered pool (hipMallocAsync on `stream`) and given
 *    back on the same stream before the call returns.  Such a call made while `stream` is being
 *    captured into a HIP graph returns CGH_EINVAL before it enqueues anything: graphs holding its
 *    allocations as memory nodes are not supported.  wasabi_hologram_fused_noalloc (and the
 *    server's jobs, whose scratch comes from their slots) allocate nothing and can be captured.
 */
#ifndef CGH_H
#define CGH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CGH_OK = 0,
    CGH_EINVAL = -1,     /* an argument is out of range or inconsistent                      */
    CGH_ENOMEM = -2,     /* device memory (or the server's memory budget) cannot hold the job */
    CGH_EHIP = -3,       /* a HIP runtime call failed                                         */
    CGH_EAGAIN = -4,     /* the result is not ready yet                                       */
    CGH_ENOTFOUND = -5,  /* unknown ticket                                                    */
    CGH_ETIMEDOUT = -6,  /* a wait timed out                                                  */
    CGH_ECANCELED = -7   /* the job was cancelled or its server destroyed                     */
} cgh_status;

enum { CGH_C64 = 0, CGH_C128 = 1 };             /* complex output type                         */
enum { CGH_F32 = 0, CGH_F16 = 1, CGH_BF16 = 2 };/* LUT value storage (rounded to nearest even) */
enum { CGH_FULL = 0, CGH_CIRC = 1 };            /* direct-sum window                           */
enum { CGH_HAAR = 0, CGH_COIF1 = 1 };           /* wavelet of the LUT                          */

/* Message of the last failing call on this thread ("" if none). */
const char *cgh_last_error(void);

/* ---------------------------------------------------------------------------------------------
 * Eq.(1): direct superposition of N point sources.
 *   pts_dev : device, n x 4 double {x, y, z, a}: metres, z > 0 (distance to the hologram plane),
 *             a = amplitude (the paper's "light intensity" a_j enters Eq.(1) linearly).
 *   window  : CGH_FULL -- every point reaches every pixel (Eq.(1) as written);
 *             CGH_CIRC -- a point reaches only the pixels inside its PSF disk,
 *             (x_h - x_j)^2 + (y_h - y_j)^2 < (z_j tan theta)^2, sin theta = lambda / (2 pitch)
 *             (the circ() support of the pre-computed PSF, Sec. 2 step 1).
 *   out_dev : device, ny rows of nx complex values, row stride ld_out elements (ld_out >= nx);
 *             overwritten.  CGH_C64: phase from FP64 r / lambda, FP32 sine/cosine, FP32 sums.
 *             CGH_C128: FP64 throughout.
 *   With CGH_CIRC and n x (tiles of 64 x 16 pixels) > 2e9 the points are binned by tile first,
 *   which synchronises `stream` once (to size the per-tile point lists); otherwise the call is
 *   fully asynchronous.
 * Errors: CGH_EINVAL (n < 0, nx/ny < 1, ld_out < nx, pitch/wavelength not > 0,
 *         wavelength >= 2 pitch, bad enum, NULL pointer with n > 0), CGH_EHIP.  n = 0 writes zeros.
 * ------------------------------------------------------------------------------------------- */
int cgh_direct(const double *pts_dev, int64_t n, int32_t nx, int32_t ny, int64_t ox, int64_t oy,
               double pitch, double wavelength, int32_t window, int32_t out_dtype, void *out_dev,
               int64_t ld_out, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Coefficient LUT (Sec. 2, step 1: pre-computation).
 * Plane d (0 <= d < n_depth) sits at z_d = z_min + (d + 1/2) dz, dz = (z_max - z_min) / n_depth.
 * Its PSF exp(i 2 pi r / lambda) circ() has radius R_d = z_d tan(theta) / pitch pixels and is
 * sampled on a W_d x W_d table centred on pixel W_d / 2, W_d = the smallest multiple of 2^(L+1)
 * with W_d >= 2 floor(R_d) + 2.  The table gets an L-level orthonormal Haar transform, and the
 * N_r(d) = ceil(gamma pi R_d^2) coefficients of largest magnitude (clamped to [1, W_d^2]; all
 * W_d^2 when gamma >= 1) are kept, values rounded to `value_dtype`.  The PSF phase and the
 * transform are computed in FP64; the ranking key is the strength |c|^2, computed in FP64 and
 * rounded to FP32, and equal keys go to the lower flat table index (row * W_d + col), so the kept
 * set is unique: any implementation of this rule keeps the same coefficients.  The LUT needs fewer
 * than 2^31 kept coefficients and fewer than 2^30 Haar blocks over all tables (else CGH_EINVAL,
 * returned before anything is allocated).
 * Phase tables (phases = 1): Eq.(2) moves a table by whole 2^L blocks, so a plane's single table
 * places only points on the 2^L grid.  With phase tables every plane gets 4^L tables, one per
 * position (sx, sy) of a point inside its 2^L x 2^L block (0 <= sx, sy < 2^L): table
 * t = d 4^L + sy 2^L + sx holds the PSF centred on pixel (W_d/2 + sx, W_d/2 + sy), with
 * W_d the smallest multiple of 2^(L+1) >= 2 floor(R_d) + 2^(L+1) so that every shifted disk fits,
 * and points are placed on any pixel.  N_r(d) is the same for the 4^L tables.  Without phase
 * tables there is one table per plane (t = d).  The LUT then takes 4^L times the memory.
 * Coiflet tables (wavelet = CGH_COIF1, the wavelet family the paper names; the order is not given
 * and the shortest, six-tap one is used): the table is transformed by the periodised orthonormal
 * filter bank lo = sqrt(2)/32 (1-s, 5+s, 14+2s, 14-2s, 1-s, -3+s), s = sqrt 7,
 * hi[n] = (-1)^n lo[5-n], along rows then columns at every level (the same Mallat layout and
 * band order as Haar), and W_d grows by 2 * 5 2^L so that no coefficient of the disk wraps round
 * the table; W_d <= 4096.  Coiflet coefficients reach beyond their 2^L block, so their holograms
 * come from wasabi_hologram only (a halo round each window, see there); wasabi_hologram_fused and
 * the server take Haar LUTs.
 * ------------------------------------------------------------------------------------------- */
typedef struct {
    double wavelength;   /* metres, 0 < wavelength < 2 pitch                                  */
    double pitch;        /* hologram sampling pitch, metres                                    */
    double z_min, z_max; /* depth range, metres, 0 < z_min < z_max                             */
    int32_t n_depth;     /* number of planes, 1 .. 65536                                       */
    int32_t levels;      /* wavelet levels L, 1 .. 6                                           */
    int32_t max_window;  /* largest allowed table side; every W_d must fit (else CGH_EINVAL),
                            and W_d / 2^L <= 65536 / (4^L + pad(L)) (the 16-bit entry keys):
                            W_d up to about 7900 (L = 3) or 4000 (L = 4) pixels               */
    int32_t value_dtype; /* CGH_F32, CGH_F16 or CGH_BF16                                       */
    double gamma;        /* selectivity, > 0                                                   */
    int32_t phases;      /* 0: one table per plane (points snapped to the 2^L grid);
                            1: 4^L phase tables per plane (points snapped to the pixel grid);
                            n_depth 4^L <= 2^20                                                */
    int32_t wavelet;     /* CGH_HAAR, or CGH_COIF1 (the coiflet of order 1, six taps)          */
} wasabi_lut_params;

typedef struct wasabi_lut wasabi_lut; /* opaque, library-owned, device-resident */

/* Build the LUT on the current device.  Synchronises `stream` once (to size the tables).
 * Errors: CGH_EINVAL, CGH_ENOMEM, CGH_EHIP.  On error *out is NULL. */
int wasabi_build_lut(const wasabi_lut_params *prm, wasabi_lut **out, void *stream);

/* Build the device LUT from host arrays in the canonical layout: table t owns entries
 * [off[t], off[t+1]) (off: n_tables + 1 int64, off[0] = 0; n_tables = n_depth, or n_depth 4^L
 * with phase tables), each an int32 flat table index idx = row * W_t + col of the table's
 * Mallat-layout coefficients (sorted ascending, no repeats) and a complex value val[2k],
 * val[2k+1] (double, rounded here to value_dtype).  The table geometry comes from `prm`; gamma is
 * ignored.  Synchronous.  Errors: CGH_EINVAL, CGH_ENOMEM, CGH_EHIP. */
int wasabi_lut_import(const wasabi_lut_params *prm, const int64_t *off_host,
                      const int32_t *idx_host, const double *val_host, wasabi_lut **out);

/* Sizes of the LUT.  Any output pointer may be NULL; per-table arrays hold n_tables values
 * (host): the plane's z, R, W and N_r of every table. */
int wasabi_lut_info(const wasabi_lut *lut, int32_t *n_tables, int64_t *total_entries,
                    int64_t *device_bytes, double *z_host, double *R_host, int32_t *W_host,
                    int64_t *Nr_host);

/* Copy the LUT to host arrays in the canonical layout above (off: n_tables + 1, idx/val: total
 * entries; val as double pairs holding the stored, rounded values).  Synchronous. */
int wasabi_lut_export(const wasabi_lut *lut, int64_t *off_host, int32_t *idx_host, double *val_host);

/* Release the LUT's device memory (waits for the device first).  NULL is accepted. */
void wasabi_lut_free(wasabi_lut *lut);

/* ---------------------------------------------------------------------------------------------
 * Points for the wavelet path.  x, y: global pixel column / row; depth: table index (the plane,
 * or with phase tables d 4^L + (y mod 2^L) 2^L + (x mod 2^L)), -1 = invalid (contributes
 * nothing); a: amplitude.  The superposition places the table at the corner of the point's 2^L
 * block (x, y floored to multiples of 2^L): exact for points on the 2^L grid and, with phase
 * tables, for any pixel.
 * ------------------------------------------------------------------------------------------- */
typedef struct {
    int32_t x, y, depth;
    float a;
} wasabi_point;

/* Depth discretisation (Sec. 2, step 1) and the 2^L position grid that makes the level-scaled
 * shift of Eq.(2) an integer: x/pitch and y/pitch go to the nearest multiple of 2^L (ties
 * upward; with phase tables to the nearest pixel, and depth is the table of the point's plane
 * and position inside its 2^L block), z to plane floor((z - z_min) / dz) (z = z_max -> the
 * last plane).  A point with z
 * outside [z_min, z_max], a non-finite value, or a snapped position beyond +-2^30 gets depth -1.
 *   pts_dev : device, n x 4 double {x, y, z, a} metres (as for cgh_direct).
 *   out_dev : device, n wasabi_point.
 * Errors: CGH_EINVAL, CGH_EHIP. */
int wasabi_quantize(const wasabi_lut *lut, const double *pts_dev, int64_t n,
                    wasabi_point *out_dev, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Eq.(2) on one sub-hologram (Sec. 2, large-scale steps 2-3): the ny x nx wavelet field psi of
 * the window whose pixel (0,0) is global pixel (ox, oy), i.e. points enter with
 * x'_j = x_j - ox, y'_j = y_j - oy.  Every kept coefficient of every valid point is added at its
 * level-scaled position; coefficients that land outside the window are dropped (exact for
 * Haar: the result equals the same window of a larger hologram).
 *   psi_dev    : device, ny x nx complex64 in Mallat layout (level-l bands of (ny>>l) x (nx>>l):
 *                H at (0, nx>>l), V at (ny>>l, 0), D at (ny>>l, nx>>l), scaling band at (0, 0)).
 *                FP32 accumulation.
 *   accumulate : 0 -- psi is overwritten with this call's field;
 *                1 -- this call's field is added to the values psi holds (one FP32 addition per
 *                coefficient), so a field can be built from several point sets in turn.
 * Requires ox, oy, nx, ny multiples of 2^L, nx, ny >= 2^L.
 * Errors: CGH_EINVAL (also accumulate not 0 or 1), CGH_ENOMEM, CGH_EHIP. */
int wasabi_superpose(const wasabi_lut *lut, const wasabi_point *pts_dev, int64_t n, int64_t ox,
                     int64_t oy, int32_t nx, int32_t ny, void *psi_dev, int32_t accumulate,
                     void *stream);

/* Inverse L-level orthonormal Haar transform (Sec. 2, step 3): psi (ny x nx complex64, Mallat
 * layout, contiguous) -> u (ny rows of nx complex64, row stride ld_u elements).
 * In place: u_dev == psi_dev with ld_u == nx overwrites the field with the hologram.  The inverse
 * moves every coefficient to pixels of another part of the field, so the in-place call first
 * copies psi to 8 nx ny bytes of scratch from the stream-ordered pool (twice the device-memory
 * traffic of the out-of-place call).  Any other overlap of u and psi is CGH_EINVAL.
 * Requires nx, ny multiples of 2^L.  Errors: CGH_EINVAL, CGH_ENOMEM (in place), CGH_EHIP. */
int wasabi_idwt(const void *psi_dev, int32_t nx, int32_t ny, int32_t levels, void *u_dev,
                int64_t ld_u, void *stream);

/* Large-scale procedure (Sec. 2, steps 2-4): the ny x nx hologram window at global (ox, oy),
 * computed as sub-holograms of at most sub x sub pixels (sub = 0: one sub-hologram), each by
 * wasabi_superpose into a scratch wavelet field followed by wasabi_idwt into its part of u.
 * With a coiflet LUT each sub-hologram's window is grown by a halo of 5 2^L pixels on every side
 * (the reach of the six-tap filters over L levels), superposed, inverted as a whole with the
 * periodised synthesis filter bank, and only its centre written to u: exact for gamma >= 1,
 * like Haar.
 *   u_dev : device, ny rows of nx complex64, row stride ld_u >= nx; overwritten.
 * Requires ox, oy, nx, ny and sub multiples of 2^L.  Errors: CGH_EINVAL, CGH_ENOMEM, CGH_EHIP. */
int wasabi_hologram(const wasabi_lut *lut, const wasabi_point *pts_dev, int64_t n, int64_t ox,
                    int64_t oy, int32_t nx, int32_t ny, int32_t sub, void *u_dev, int64_t ld_u,
                    void *stream);

/* Same result as wasabi_hologram, computed tile by tile: each tile's Haar blocks are superposed
 * (Eq.(2)) and inverted (Sec. 2, step 3) inside on-chip memory, so the wavelet field never goes
 * to device memory.  Exact reordering for Haar, whose 2^L x 2^L blocks are independent.
 * Same arguments and errors as wasabi_hologram without `sub`; a coiflet LUT gives CGH_EINVAL
 * (its coefficients reach beyond the tile's blocks). */
int wasabi_hologram_fused(const wasabi_lut *lut, const wasabi_point *pts_dev, int64_t n,
                          int64_t ox, int64_t oy, int32_t nx, int32_t ny, void *u_dev,
                          int64_t ld_u, void *stream);

/* wasabi_hologram_fused for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, result and
 * errors as wasabi_hologram_fused; nothing is allocated and no memory is freed: the binning's
 * scratch comes from a static device buffer of 64 MiB that the library holds on every device it
 * runs on until the process ends (a problem needing more gives CGH_ENOMEM before any launch;
 * enough for the 2048 x 2048, N = 10^4 workload, about 16 MiB).  Every call on a device shares
 * that device's buffer: calls that overlap in time on one device (other streams, other threads)
 * race and must be serialised by the caller; calls on one stream are ordered by it.  Counters in
 * the buffer are cleared by the call's own kernels. */
int wasabi_hologram_fused_noalloc(const wasabi_lut *lut, const wasabi_point *pts_dev, int64_t n,
                                  int64_t ox, int64_t oy, int32_t nx, int32_t ny, void *u_dev,
                                  int64_t ld_u, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Numerical propagation (the reconstruction Sec. 3 assesses holograms by) and the wavefront
 * recording plane (the conclusion's next step).
 *
 * cgh_propagate: angular-spectrum propagation of a complex field by `distance` metres (either
 * sign), the field taken as periodic: u_out = IFFT2(FFT2(u_in) H) with
 * H(fx, fy) = exp(i 2 pi distance sqrt(1/lambda^2 - fx^2 - fy^2)) where fx^2 + fy^2 < 1/lambda^2,
 * 0 elsewhere; fx = k / (nx pitch), fy = k / (ny pitch), k in FFT order (0 .. n/2-1, -n/2 .. -1).
 *   u_in, u_out : device, ny x nx complex64 row-major, contiguous; u_out may equal u_in.
 *   nx, ny      : powers of two in [64, 8192].
 * FP32 transforms; twiddles and the transfer function's phase from FP64 angles.  Takes 16 nx ny
 * bytes of scratch from the stream-ordered pool.  Errors: CGH_EINVAL, CGH_ENOMEM, CGH_EHIP.
 *
 * wasabi_hologram_wrp: the hologram of points far from the hologram plane through a wavefront
 * recording plane z_wrp metres from it.  Every point's depth is taken from the WRP (z - z_wrp,
 * which must lie in the LUT's [z_min, z_max]; others contribute nothing), WASABI computes the
 * field on the WRP (as wasabi_quantize + wasabi_hologram_fused at origin (0, 0)), and
 * cgh_propagate carries it over z_wrp to the hologram plane, in place in u (a coiflet LUT's WRP
 * field comes from wasabi_hologram instead of the fused path).
 *   pts_dev : device, n x 4 double {x, y, z, a} metres (as for wasabi_quantize).
 *   u_dev   : device, ny x nx complex64 row-major, contiguous; overwritten.
 *   nx, ny  : powers of two in [64, 8192].
 * Errors: CGH_EINVAL, CGH_ENOMEM, CGH_EHIP. */
int cgh_propagate(const void *u_in_dev, void *u_out_dev, int32_t nx, int32_t ny, double distance,
                  double pitch, double wavelength, void *stream);
int wasabi_hologram_wrp(const wasabi_lut *lut, const double *pts_dev, int64_t n, double z_wrp,
                        int32_t nx, int32_t ny, void *u_dev, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Hologram server: a queue of hologram jobs served with continuous batching.
 *
 * Every job is one hologram (Sec. 2): its points are snapped (wasabi_quantize) and superposed and
 * inverted tile by tile (wasabi_hologram_fused) with the server's shared LUT into a
 * ny x nx complex64 hologram owned by the server.  Up to max_slots jobs run at once, each on a
 * stream of its own, so the work of different jobs overlaps on the device; a job is admitted
 * (strictly in submission order) as soon as a slot is free and its memory fits the budget, also
 * while others run.  The budget counts the device memory the jobs hold: the shared LUT (charged
 * once, at creation), each job's result (8 nx ny bytes, held until cgh_server_release) and each
 * slot's arena, which holds the working memory of the job running in it (device points,
 * quantised points, the superposition's scratch), is kept for the slot's next job, grows for a
 * larger one and is given back when an idle slot's share is needed to admit a job.
 * A scheduler thread owned by the server issues the work; the calls below are thread-safe.
 * Each slot is a stream: keep max_slots + the caller's own streams within the device's hardware
 * queues per process (GPU_MAX_HW_QUEUES, 4 by default), or enqueue calls start to wait on each
 * other; 2-3 slots overlap one job's host-side issue with the device work of others.
 * Times are seconds on a monotonic host clock since the server was created.
 * ------------------------------------------------------------------------------------------- */
typedef struct cgh_server cgh_server; /* opaque */

typedef struct {
    size_t hbm_budget_bytes;   /* device memory the jobs may hold together (> 0)                  */
    int32_t max_slots;         /* jobs running at once, 1 .. 64                                   */
    int32_t simulate;          /* 0: run on the device of `lut`.  1: host model, no device work:
                                  a job "runs" for sim_ns_per_pixel * nx * ny ns (for testing the
                                  admission policy without a GPU; results have u = NULL)          */
    double sim_ns_per_pixel;
    const wasabi_lut *lut;     /* shared by every job; must outlive the server (ignored when
                                  simulate = 1 and NULL is given: jobs then need multiples of 8)  */
    uint64_t fail_ticket;      /* testing the failure path: the job with this ticket fails as its
                                  work is being issued (after its result memory was taken), with
                                  status CGH_EHIP; 0 = none                                       */
} cgh_server_config;

typedef struct {
    const double *host_pts; /* host, n x 4 double {x, y, z, a} metres as for wasabi_quantize;
                               copied by cgh_server_submit (the caller may reuse it at once)      */
    int64_t n;              /* 0 .. 2^31 - 1                                                      */
    int32_t nx, ny;         /* hologram size, positive multiples of 2^L, at most 65536 each       */
} cgh_job;

typedef struct {
    const void *u;          /* device, ny x nx complex64 row-major, valid until release; NULL for
                               a cancelled or failed job and in simulation                        */
    int32_t nx, ny;
    double t_submit, t_admit, t_start, t_done; /* submit call, admission, all work enqueued on the
                                                  job's stream, work seen done                    */
    double gpu_ms;          /* device time of the job's work (HIP events on its stream)           */
    int32_t status;         /* CGH_OK, CGH_ECANCELED, or the error code of the failed job         */
    int32_t slot;           /* slot (stream) that ran it, -1 if it never ran                      */
} cgh_result;

typedef struct {
    int64_t submitted, completed, canceled, failed; /* jobs by final state (completed = OK)       */
    int64_t queued, running;                        /* now                                        */
    int64_t max_running;                            /* most jobs running at once so far           */
    size_t bytes_in_use, peak_bytes;                /* budgeted bytes now / at most so far        */
    size_t arena_bytes;                             /* of bytes_in_use: the slots' arenas         */
    size_t lut_bytes;                               /* of bytes_in_use: the shared LUT            */
} cgh_server_stats;

/* Create a server on the current device (the LUT's).  Errors: CGH_EINVAL (NULL arguments, budget 0,
 * max_slots out of range, LUT on another device), CGH_ENOMEM (the LUT alone fills the budget),
 * CGH_EHIP. */
int cgh_server_create(const cgh_server_config *cfg, cgh_server **out);

/* Queue a job; *ticket identifies it (> 0).  Errors: CGH_EINVAL (bad sizes, NULL points with
 * n > 0), CGH_ENOMEM (the job alone exceeds the budget, or host staging memory failed),
 * CGH_ECANCELED (the server is shutting down), CGH_EHIP. */
int cgh_server_submit(cgh_server *srv, const cgh_job *job, uint64_t *ticket);

/* Wait until the job has ended (done, failed or cancelled) and describe it in *out.  timeout_ms < 0
 * waits without limit.  Returns CGH_OK when the job has ended (its own outcome is out->status),
 * CGH_ETIMEDOUT, CGH_ENOTFOUND (unknown or released ticket), CGH_ECANCELED (server destroyed
 * while waiting). */
int cgh_server_wait(cgh_server *srv, uint64_t ticket, int32_t timeout_ms, cgh_result *out);

/* Cancel a queued or running job: a queued job ends at once, a running one when its device work
 * ends (that work is not interrupted); either way it ends with status CGH_ECANCELED and holds no
 * memory.  Errors: CGH_ENOTFOUND, CGH_EINVAL (the job has already ended: release it instead). */
int cgh_server_cancel(cgh_server *srv, uint64_t ticket);

/* Forget an ended job and give its result memory back to the budget.  The result buffer is freed
 * in the order of the job's own stream only, and the server may hand the memory to its next job
 * at once: the caller must therefore have finished (synchronised) every stream whose device work
 * reads the result before calling this.  Errors: CGH_ENOTFOUND, CGH_EAGAIN (the job has not ended
 * yet). */
int cgh_server_release(cgh_server *srv, uint64_t ticket);

/* Current counters.  Errors: CGH_EINVAL. */
int cgh_server_query(cgh_server *srv, cgh_server_stats *out);

/* Cancel the queued jobs, wait for the running ones, wake every waiter (CGH_ECANCELED) and free the
 * server with all results.  No other call may use `srv` once this returns.  NULL is accepted. */
int cgh_server_destroy(cgh_server *srv);

/* ---------------------------------------------------------------------------------------------
 * Kernel tracing.  While enabled, the library records a pair of HIP events on the launching
 * stream around each of its kernels (or kernel groups), under these names:
 *   "direct", "quantize", "psf_haar", "select", "bin" (count + scan + fill), "tile_superpose",
 *   "tile_fused", "idwt".
 * cgh_profile_query synchronises the recorded events and returns the summed elapsed time and the
 * number of launches for `name` (0 / 0 if none).  Not for concurrent use from several threads.
 * ------------------------------------------------------------------------------------------- */
int cgh_profile_enable(int32_t on);
int cgh_profile_reset(void);
int cgh_profile_query(const char *name, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* CGH_H */
