// Error state, stream-ordered scratch and plane geometry of libcgh.so.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "common.hpp"

namespace cgh {

static thread_local char g_msg[1024] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return code;
}

Scratch::~Scratch()
{
    for (void *p : ptrs_) (void)hipFreeAsync(p, stream_);
}

int Scratch::alloc(void **p, size_t bytes)
{
    *p = nullptr;
    if (arena_) {
        const size_t b = std::max<size_t>((bytes + 255) & ~(size_t)255, 256);
        if (used_ + b > cap_) return fail(CGH_ENOMEM, "scratch arena of %zu bytes exhausted", cap_);
        *p = arena_ + used_;
        used_ += b;
        return CGH_OK;
    }
    if (!capture_checked_) {
        // Under stream capture the allocations and frees below would become graph memory nodes;
        // replaying such a graph has crashed the host process here, so a capturing caller is
        // refused before anything is enqueued (every call allocates before its first launch).
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        const hipError_t ce = hipStreamIsCapturing(stream_, &st);
        if (ce != hipSuccess) return fail(CGH_EHIP, "hipStreamIsCapturing: %s", hipGetErrorString(ce));
        if (st != hipStreamCaptureStatusNone)
            return fail(CGH_EINVAL, "this call allocates stream-ordered scratch and cannot be captured into a HIP "
                                    "graph; wasabi_hologram_fused_noalloc can");
        capture_checked_ = true;
    }
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMallocAsync(p, bytes, stream_);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        return fail(CGH_ENOMEM, "scratch allocation of %zu bytes failed", bytes);
    }
    if (e != hipSuccess) return fail(CGH_EHIP, "hipMallocAsync: %s", hipGetErrorString(e));
    ptrs_.push_back(*p);
    return CGH_OK;
}

int prepare_pool()
{
    static std::mutex mu;
    static std::vector<int> done;
    int dev = 0;
    CGH_TRY_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    for (int d : done)
        if (d == dev) return CGH_OK;
    hipMemPool_t pool;
    CGH_TRY_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
    uint64_t thr = UINT64_MAX;
    CGH_TRY_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr));
    // Memory freed on one stream is reused by another only once its work has finished: the pool
    // must not make one stream wait for another (work on different streams stays independent).
    int no = 0;
    CGH_TRY_HIP(hipMemPoolSetAttribute(pool, hipMemPoolReuseAllowInternalDependencies, &no));
    done.push_back(dev);
    return CGH_OK;
}

// ---- kernel tracing ---------------------------------------------------------------------------
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof;

ProfScope::ProfScope(const char *name, hipStream_t s) : name_(name), s_(s)
{
    if (!g_prof_on) return;
    if (hipEventCreate(&a_) != hipSuccess || hipEventRecord(a_, s_) != hipSuccess) {
        (void)hipGetLastError();
        if (a_) (void)hipEventDestroy(a_);
        a_ = nullptr;
    }
}

ProfScope::~ProfScope()
{
    if (!a_) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) != hipSuccess || hipEventRecord(b, s_) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventDestroy(a_);
        if (b) (void)hipEventDestroy(b);
        return;
    }
    std::lock_guard<std::mutex> lock(g_prof_mu);
    g_prof.push_back(ProfRec{name_, a_, b});
}

int validate_params(const wasabi_lut_params *prm)
{
    if (!prm) return fail(CGH_EINVAL, "params is NULL");
    if (!(prm->pitch > 0) || !(prm->wavelength > 0) || !(prm->wavelength < 2 * prm->pitch))
        return fail(CGH_EINVAL, "need 0 < wavelength < 2 * pitch");
    if (!(prm->z_min > 0) || !(prm->z_max > prm->z_min) || !std::isfinite(prm->z_max))
        return fail(CGH_EINVAL, "need 0 < z_min < z_max");
    if (prm->n_depth < 1 || prm->n_depth > 65536) return fail(CGH_EINVAL, "n_depth out of range");
    if (prm->levels < 1 || prm->levels > 6) return fail(CGH_EINVAL, "levels must be 1..6");
    if (prm->value_dtype < CGH_F32 || prm->value_dtype > CGH_BF16)
        return fail(CGH_EINVAL, "unknown value_dtype");
    if (!(prm->gamma > 0) || !std::isfinite(prm->gamma)) return fail(CGH_EINVAL, "gamma must be > 0");
    if (prm->phases != 0 && prm->phases != 1) return fail(CGH_EINVAL, "phases must be 0 or 1");
    if (prm->wavelet != CGH_HAAR && prm->wavelet != CGH_COIF1) return fail(CGH_EINVAL, "unknown wavelet");
    if (prm->phases && ((int64_t)prm->n_depth << (2 * prm->levels)) > (INT64_C(1) << 20))
        return fail(CGH_EINVAL, "n_depth * 4^L phase tables exceed 2^20");
    return CGH_OK;
}

// Sec. 2, step 1: planes at the centres of n_depth equal depth cells; PSF radius from the
// largest diffraction angle of the pitch (sin theta = lambda / 2p); table side W_d the smallest
// multiple of 2^(L+1) holding the disk (so the table centre is on the 2^L grid; with phase tables
// the disk around any centre shifted by less than 2^L pixels right / down); N_r = gamma pi R^2.
// With phase tables each plane's values repeat for its 4^L tables.
int lut_geometry(wasabi_lut *lut)
{
    const wasabi_lut_params &p = lut->prm;
    const int n = p.n_depth;
    const double sin_t = p.wavelength / (2.0 * p.pitch);
    const double tan_t = sin_t / std::sqrt(1.0 - sin_t * sin_t);
    const double dz = (p.z_max - p.z_min) / (double)n;
    const int q = 1 << (p.levels + 1);
    const int B = 1 << p.levels;
    const int key_room = 65536 / block_stride(p.levels);  // blocks per row that keys can address
    lut->P = p.phases ? 1 << (2 * p.levels) : 1;
    lut->n_tables = n * lut->P;
    const int P = lut->P, nt = lut->n_tables;
    // The superposition addresses entries with 32-bit integers and per-block offsets with 32-bit byte
    // offsets: both totals are bounded here, before anything is allocated.
    int64_t blk_total = 0, entries = 0;
    lut->z.resize(nt);
    lut->R.resize(nt);
    lut->W.resize(nt);
    lut->Nr.resize(nt);
    for (int d = 0; d < n; d++) {
        const double z = p.z_min + ((double)d + 0.5) * dz;
        const double R = z * tan_t / p.pitch;
        if (!(R < 1e6)) return fail(CGH_EINVAL, "plane %d: PSF radius too large", d);
        // coiflet tables: a margin of 5 2^L pixels on each side keeps the disk's coefficients from
        // wrapping round the periodised transform
        const int64_t need = 2 * (int64_t)std::floor(R) + (p.phases ? q : 2) +
                             (p.wavelet == CGH_COIF1 ? 2 * 5 * B : 0);
        const int64_t W = ((need + q - 1) / q) * q;
        if (W > p.max_window)
            return fail(CGH_EINVAL, "plane %d needs a %lld-pixel table > max_window %d", d,
                        (long long)W, p.max_window);
        if (p.wavelet == CGH_COIF1 && W > 4096)
            return fail(CGH_EINVAL, "plane %d: coiflet table side %lld > 4096", d, (long long)W);
        if (W / B > key_room)
            return fail(CGH_EINVAL, "plane %d: table side %lld too large for L=%d", d,
                        (long long)W, p.levels);
        const int64_t all = W * W;
        int64_t nr;
        if (p.gamma >= 1.0) {
            nr = all;
        } else {
            nr = (int64_t)std::ceil(p.gamma * M_PI * R * R);
            if (nr < 1) nr = 1;
            if (nr > all) nr = all;
        }
        blk_total += (int64_t)P * ((W / B) * (W / B) + 1);
        entries += (int64_t)P * nr;
        if (blk_total >= (INT64_C(1) << 30))
            return fail(CGH_EINVAL, "LUT of 2^30 or more Haar blocks (%d tables of up to %lld^2 pixels)", nt,
                        (long long)W);
        if (entries >= INT32_MAX)
            return fail(CGH_EINVAL, "LUT of more than 2^31 - 1 kept coefficients");
        for (int t = d * P; t < (d + 1) * P; ++t) {
            lut->z[t] = z;
            lut->R[t] = R;
            lut->W[t] = (int32_t)W;
            lut->Nr[t] = nr;
        }
    }
    return CGH_OK;
}

// Analysis filter bank of the LUT's wavelet: Haar (1, 1)/sqrt 2, or the coiflet of order 1 from its
// closed form lo = sqrt(2)/32 (1-s, 5+s, 14+2s, 14-2s, 1-s, -3+s), s = sqrt 7 (Daubechies, Ten Lectures
// on Wavelets, Sec. 8.2); hi[n] = (-1)^n lo[taps-1-n].  Returns the number of taps.
int wavelet_filters(int wavelet, double *lo, double *hi)
{
    int taps;
    if (wavelet == CGH_COIF1) {
        const double s = std::sqrt(7.0), c = std::sqrt(2.0) / 32.0;
        const double f[6] = {1 - s, 5 + s, 14 + 2 * s, 14 - 2 * s, 1 - s, -3 + s};
        taps = 6;
        for (int n = 0; n < taps; ++n) lo[n] = c * f[n];
    } else {
        taps = 2;
        lo[0] = lo[1] = 1.0 / std::sqrt(2.0);
    }
    for (int n = 0; n < taps; ++n) hi[n] = ((n & 1) ? -1.0 : 1.0) * lo[taps - 1 - n];
    return taps;
}

}  // namespace cgh

extern "C" const char *cgh_last_error(void) { return cgh::g_msg; }

extern "C" int cgh_profile_enable(int32_t on)
{
    cgh::g_prof_on = on != 0;
    return CGH_OK;
}

extern "C" int cgh_profile_reset(void)
{
    std::lock_guard<std::mutex> lock(cgh::g_prof_mu);
    for (auto &r : cgh::g_prof) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    cgh::g_prof.clear();
    return CGH_OK;
}

extern "C" int cgh_profile_query(const char *name, double *total_ms, int64_t *launches)
{
    using namespace cgh;
    if (!name || !total_ms || !launches) return fail(CGH_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(g_prof_mu);
    double t = 0.0;
    int64_t k = 0;
    for (auto &r : g_prof) {
        if (r.name != name) continue;
        CGH_TRY_HIP(hipEventSynchronize(r.b));
        float ms = 0.0f;
        CGH_TRY_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        t += ms;
        ++k;
    }
    *total_ms = t;
    *launches = k;
    return CGH_OK;
}
