// host_common.h -- host-side support shared by the library's entry points: error
// reporting, the device check, configuration checks and optional event timing.
#ifndef COMET_HOST_COMMON_H
#define COMET_HOST_COMMON_H

#include <hip/hip_runtime.h>

#include <stddef.h>

#include "comet.h"

namespace chost {

// Records a formatted message for comet_last_error() and returns `status`.
int fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
// Clears / returns the calling thread's last error message.
void clear_error();
const char *last_error();
// COMET_OK when the current device is gfx950 (cached per device).
int check_device();
// COMET_EHIP with details when the last kernel launch failed.
int launched(const char *what);
// Checks every field of a comet_config.
int check_config(const comet_config *cfg);
bool finite_pos(double v);
size_t align256(size_t v);
// Checks a comet_field (not the map's values): b set, nx, ny, nz >= 2, stepper 0 or 1,
// finite origin, spacings > 0.
int check_field(const char *who, const comet_field *field);
// Launches the field map's track recording (one thread per seed); rho, when set,
// receives the track's chunk radii [window][S] taken while recording.
int launch_field_record(const double *seeds6, int64_t S, const comet_field *field,
                        double charge, double h, int K, double *track, double *rho,
                        hipStream_t stream);

// Kernel kinds for comet_profile_end().
enum { kProfTrack = 0, kProfDca = 1, kProfSum = 2, kProfSelect = 3 };

// While profiling is on: a device counter (current device) that the DCA scans add
// their (seed, wire, point) distance evaluations to; nullptr otherwise.
unsigned long long *scan_counter();

// Brackets the launches made during its lifetime with two HIP events on `stream`
// when profiling is on (comet_profile_begin) and `enabled`; does nothing otherwise.
class ProfScope {
  public:
    ProfScope(int kind, hipStream_t stream, bool enabled = true);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;

  private:
    hipStream_t stream_;
    int kind_;
    hipEvent_t start_ = nullptr, stop_ = nullptr;
};

}  // namespace chost

#endif  // COMET_HOST_COMMON_H
