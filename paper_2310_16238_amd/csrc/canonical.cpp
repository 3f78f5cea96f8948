// canonical.cpp -- see canonical.h.
#include "canonical.h"

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace coxmi {

namespace {
struct Key {
    int32_t s;
    double t;
    int64_t i;
};
}  // namespace

void canonical_order(int64_t n, const double *time, const uint8_t *event, const int32_t *stratum,
                     std::vector<int64_t> &perm, std::vector<uint32_t> &meta)
{
    // sort packed keys (no indirect loads in the comparator)
    std::vector<Key> k((size_t)n);
    for (int64_t i = 0; i < n; ++i) k[i] = Key{stratum ? stratum[i] : 0, time[i], i};
    std::sort(k.begin(), k.end(), [](const Key &a, const Key &b) {
        if (a.s != b.s) return a.s < b.s;
        if (a.t != b.t) return a.t > b.t;
        return a.i < b.i;
    });
    perm.resize((size_t)n);
    meta.assign((size_t)n, 0u);
    uint32_t gcount = 0;
    for (int64_t i = 0; i < n; ++i) {
        perm[i] = k[i].i;
        const bool new_stratum = i == 0 || k[i].s != k[i - 1].s;
        if (new_stratum || k[i].t != k[i - 1].t) gcount = 0;
        if (new_stratum) meta[i] |= kHeadBit;
        if (event[k[i].i]) {
            meta[i] |= kEventBit;
            ++gcount;
        }
        const bool last_of_group = i + 1 == n || k[i + 1].s != k[i].s || k[i + 1].t != k[i].t;
        if (last_of_group) meta[i] |= gcount;
    }
}

const char *check_data(int64_t n, int64_t p, int64_t ldx, const double *x, const double *time,
                       const uint8_t *event)
{
    if (n < 1 || p < 1) return "need n >= 1 and p >= 1";
    if (ldx < n) return "ldx < n";
    if (!x || !time || !event) return "x, time and event are required";
    if (n > (int64_t)kCountMask) return "n exceeds 2^29 - 1";
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(time[i])) return "time contains NaN or inf";
        if (event[i] > 1) return "event must be 0 or 1";
    }
    return nullptr;
}

}  // namespace coxmi
