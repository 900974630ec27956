// lbmax_checks.h -- host-side checks of readout values (plain C++, no HIP):
// the finite check behind LB_ENONFINITE and the lattice Mach guard behind
// LB_WARN_MACH.  Used by lbmax_runtime.hip; also compiled alone by the CPU
// tests.
#pragma once

#include <cmath>
#include <cstddef>

namespace lbmax {

// The lattice speed of sound is 1/sqrt(3) (D2Q9, Sec. III); the BGK scheme
// reproduces Navier-Stokes only at small Mach number.  |u| above 0.1 (Mach
// 0.17) raises the guard.
constexpr double kMachGuardSpeed = 0.1;

struct ValueScan {
    size_t nonfinite = 0;  // NaN or infinite entries
    double max_abs = 0.0;  // largest finite magnitude
};

inline ValueScan scan_values(const double *a, size_t n)
{
    ValueScan r;
    for (size_t i = 0; i < n; ++i) {
        const double v = a[i];
        if (!std::isfinite(v)) {
            ++r.nonfinite;
            continue;
        }
        const double m = std::fabs(v);
        if (m > r.max_abs)
            r.max_abs = m;
    }
    return r;
}

// Largest speed |u| over n nodes of a velocity field (ux, uy may be null:
// that component is taken as zero).
inline double max_speed(const double *ux, const double *uy, size_t n)
{
    double m = 0.0;
    for (size_t i = 0; i < n; ++i) {
        const double x = ux ? ux[i] : 0.0, y = uy ? uy[i] : 0.0;
        const double s = std::sqrt(x * x + y * y);
        if (std::isnan(s) || s > m)
            m = s;  // a NaN speed is kept: it trips the guard
    }
    return m;
}

inline bool mach_guard_trips(double speed) { return !(speed <= kMachGuardSpeed); }

}  // namespace lbmax
