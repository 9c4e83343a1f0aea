// The CIL statistic's range, radii and bins left on the device for one
// read-back at the end of a longer chain (distance.hip, api.hip).
#pragma once

namespace cil {

// Range and radii as the device formed them: the canonical extremes of the
// range candidates, the candidates' statistics, a status (0 ok, 1 degenerate
// range, 2 a non-finite distance, 3 candidate-list overflow) and the ladder.
struct RangeOut {
    double d2min, d2max;
    long long nrange, nrange_exact;
    int status, pad;
    double radii[256];
};

// The histogram [M + 1], the re-check list counters (listed pairs, exact
// fallbacks), the list capacity and the range (device).
struct AsyncBins {
    unsigned long long *hist = nullptr;
    unsigned long long *nlist = nullptr;
    long long cap = 0;
    long long nrange = 0, nrange_exact = 0;
    RangeOut *ro = nullptr;
};

}  // namespace cil
