// runtime.hip -- host-side support shared by every entry point of the library:
// error reporting, the device check, configuration checks and the optional
// per-kernel event timing (comet_profile_begin / comet_profile_end).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "comet.h"
#include "host_common.h"

namespace chost {

namespace {
thread_local char g_last_error[512] = "";

struct ProfRecord {
    hipEvent_t start, stop;
    int kind;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof_records;
std::vector<hipEvent_t> g_prof_pool;
unsigned long long *g_scan_counter[64] = {};  // per device, allocated on first use
int g_scan_dev = -1;                          // device of the running count
long long g_scan_points = 0;                  // the last finished count

// An event from the pool, or a new one (caller holds g_prof_mu).
hipEvent_t prof_event()
{
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}
}  // namespace

int fail(int status, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return status;
}

void clear_error() { g_last_error[0] = 0; }

const char *last_error() { return g_last_error; }

int check_device()
{
    static std::mutex mu;
    static int cached[64];  // 0 unknown, 1 gfx950, -1 other
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(COMET_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= 64)
        return fail(COMET_EUNSUPPORTED, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (cached[dev] == 0) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess)
            return fail(COMET_EHIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
        cached[dev] = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
        if (cached[dev] < 0)
            return fail(COMET_EUNSUPPORTED, "device %d is %s, not gfx950", dev, prop.gcnArchName);
    }
    if (cached[dev] < 0)
        return fail(COMET_EUNSUPPORTED, "device %d is not gfx950", dev);
    return COMET_OK;
}

int launched(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(COMET_EHIP, "%s launch: %s", what, hipGetErrorString(e));
    return COMET_OK;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

int check_field(const char *who, const comet_field *field)
{
    if (!field || !field->b)
        return fail(COMET_EINVAL, "%s: NULL field map", who);
    if (field->nx < 2 || field->ny < 2 || field->nz < 2 ||
        (field->stepper != 0 && field->stepper != 1) ||
        !finite_pos(field->dx) || !finite_pos(field->dy) || !finite_pos(field->dz) ||
        !isfinite(field->x0) || !isfinite(field->y0) || !isfinite(field->z0))
        return fail(COMET_EINVAL, "%s: need nx, ny, nz >= 2, stepper 0 or 1, finite origin, "
                                  "spacings > 0", who);
    return COMET_OK;
}

unsigned long long *scan_counter()
{
    std::lock_guard<std::mutex> lock(g_prof_mu);
    int dev = -1;
    if (!g_prof_on || hipGetDevice(&dev) != hipSuccess || dev != g_scan_dev)
        return nullptr;
    return g_scan_counter[dev];
}

int check_config(const comet_config *cfg)
{
    if (!cfg)
        return fail(COMET_EINVAL, "cfg is NULL");
    if (!isfinite(cfg->bz_tesla) || !isfinite(cfg->charge_e))
        return fail(COMET_EINVAL, "bz_tesla and charge_e must be finite");
    if (!finite_pos(cfg->step_mm))
        return fail(COMET_EINVAL, "step_mm must be finite and > 0");
    if (cfg->n_steps < 1 || cfg->n_steps > (1 << 24))
        return fail(COMET_EINVAL, "n_steps must be in [1, 2^24]");
    if (!finite_pos(cfg->lambda_mm))
        return fail(COMET_EINVAL, "lambda_mm must be finite and > 0");
    if (cfg->reserved != 0)
        return fail(COMET_EINVAL, "reserved must be 0");
    return COMET_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

ProfScope::ProfScope(int kind, hipStream_t stream, bool enabled) : stream_(stream), kind_(kind)
{
    if (!enabled)
        return;
    std::lock_guard<std::mutex> lock(g_prof_mu);
    if (!g_prof_on)
        return;
    start_ = prof_event();
    stop_ = prof_event();
    if (start_ && stop_)
        (void)hipEventRecord(start_, stream_);
}

ProfScope::~ProfScope()
{
    if (!start_ || !stop_)
        return;
    (void)hipEventRecord(stop_, stream_);
    std::lock_guard<std::mutex> lock(g_prof_mu);
    g_prof_records.push_back({start_, stop_, kind_});
}

}  // namespace chost

extern "C" {

const char *comet_last_error(void) { return chost::last_error(); }

int comet_profile_begin(void)
{
    using namespace chost;
    std::lock_guard<std::mutex> lock(g_prof_mu);
    for (auto &r : g_prof_records) {
        g_prof_pool.push_back(r.start);
        g_prof_pool.push_back(r.stop);
    }
    g_prof_records.clear();
    g_scan_dev = -1;
    g_scan_points = 0;
    int dev = -1;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) {
        if (!g_scan_counter[dev] &&
            hipMalloc((void **)&g_scan_counter[dev], sizeof(unsigned long long)) != hipSuccess)
            g_scan_counter[dev] = nullptr;
        if (g_scan_counter[dev] &&
            hipMemset(g_scan_counter[dev], 0, sizeof(unsigned long long)) == hipSuccess)
            g_scan_dev = dev;
    }
    g_prof_on = true;
    return COMET_OK;
}

int comet_profile_end(double ms[COMET_PROFILE_KINDS], int64_t launches[COMET_PROFILE_KINDS])
{
    using namespace chost;
    std::lock_guard<std::mutex> lock(g_prof_mu);
    g_prof_on = false;
    int status = COMET_OK;
    for (int k = 0; k < COMET_PROFILE_KINDS; ++k) {
        if (ms)
            ms[k] = 0.0;
        if (launches)
            launches[k] = 0;
    }
    for (auto &r : g_prof_records) {
        float t = 0.0f;
        hipError_t e = hipEventSynchronize(r.stop);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&t, r.start, r.stop);
        if (e != hipSuccess) {
            status = fail(COMET_EHIP, "comet_profile_end: %s", hipGetErrorString(e));
        } else if (r.kind >= 0 && r.kind < COMET_PROFILE_KINDS) {
            if (ms)
                ms[r.kind] += t;
            if (launches)
                launches[r.kind] += 1;
        }
        g_prof_pool.push_back(r.start);
        g_prof_pool.push_back(r.stop);
    }
    g_prof_records.clear();
    if (g_scan_dev >= 0) {
        unsigned long long n = 0;
        int cur = -1;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(g_scan_dev);
        hipError_t e = hipMemcpy(&n, g_scan_counter[g_scan_dev], sizeof(n), hipMemcpyDeviceToHost);
        (void)hipSetDevice(cur);
        if (e != hipSuccess && status == COMET_OK)
            status = fail(COMET_EHIP, "comet_profile_end: %s", hipGetErrorString(e));
        g_scan_points = (long long)n;
        g_scan_dev = -1;
    }
    return status;
}

int comet_profile_scan_points(int64_t *points)
{
    using namespace chost;
    if (!points)
        return fail(COMET_EINVAL, "comet_profile_scan_points: NULL pointer");
    std::lock_guard<std::mutex> lock(g_prof_mu);
    *points = g_scan_points;
    return COMET_OK;
}

}  // extern "C"
