// canonical.cpp -- see canonical.h.
#include "canonical.h"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace coxmi {

namespace {

// Order-preserving image of a time for a descending sort: larger times get
// smaller keys; -0 and +0 are the same time.  Times are finite (checked).
inline uint64_t desc_key(double t)
{
    if (t == 0.0) t = 0.0;
    uint64_t u;
    std::memcpy(&u, &t, sizeof u);
    u = (u >> 63) ? ~u : (u | 0x8000000000000000ull);   // ascending order of t
    return ~u;
}

struct KI {
    uint64_t k;
    int64_t i;
};

// Stable LSD radix sort of a[0, n) by k (8-bit digits; a digit on which all
// keys agree is skipped).  tmp: scratch of n elements.
void radix_by_key(KI *a, KI *tmp, int64_t n)
{
    for (int shift = 0; shift < 64; shift += 8) {
        int64_t cnt[257] = {0};
        for (int64_t r = 0; r < n; ++r) ++cnt[((a[r].k >> shift) & 0xff) + 1];
        bool trivial = false;
        for (int d = 1; d <= 256; ++d) trivial |= cnt[d] == n;
        if (trivial) continue;
        for (int d = 1; d <= 256; ++d) cnt[d] += cnt[d - 1];
        for (int64_t r = 0; r < n; ++r) tmp[cnt[(a[r].k >> shift) & 0xff]++] = a[r];
        std::memcpy(a, tmp, sizeof(KI) * (size_t)n);
    }
}

// Stable sort of a[0, n) by k.
void sort_by_key(KI *a, KI *tmp, int64_t n)
{
    if (n <= 32) {   // insertion sort
        for (int64_t r = 1; r < n; ++r) {
            const KI v = a[r];
            int64_t q = r - 1;
            while (q >= 0 && a[q].k > v.k) {
                a[q + 1] = a[q];
                --q;
            }
            a[q + 1] = v;
        }
    } else if (n <= 4096) {   // indices ascend on entry, so (k, i) order is the stable order
        std::sort(a, a + n, [](const KI &x, const KI &y) { return x.k != y.k ? x.k < y.k : x.i < y.i; });
    } else {
        radix_by_key(a, tmp, n);
    }
}

}  // namespace

void canonical_order(int64_t n, const double *time, const uint8_t *event, const int32_t *stratum,
                     std::vector<int64_t> &perm, std::vector<uint32_t> &meta)
{
    // 1. rows grouped by stratum (ascending label), original order kept inside a stratum
    std::vector<KI> a((size_t)n), tmp((size_t)n);
    std::vector<int64_t> seg;   // start of each stratum's run in a, then n
    if (!stratum) {
        for (int64_t r = 0; r < n; ++r) a[r] = KI{0, r};
        seg = {0, n};
    } else {
        int32_t lo = stratum[0], hi = stratum[0];
        for (int64_t r = 1; r < n; ++r) {
            lo = std::min(lo, stratum[r]);
            hi = std::max(hi, stratum[r]);
        }
        const int64_t range = (int64_t)hi - (int64_t)lo + 1;
        if (range <= 2 * n + 1024) {   // counting sort on the label
            std::vector<int64_t> start((size_t)range + 1, 0);   // start[c]: first position of label lo + c
            for (int64_t r = 0; r < n; ++r) ++start[(size_t)((int64_t)stratum[r] - lo) + 1];
            for (int64_t c = 0; c < range; ++c) {
                if (start[c + 1] > 0) seg.push_back(start[c]);   // a label that occurs
                start[c + 1] += start[c];
            }
            for (int64_t r = 0; r < n; ++r) a[start[(size_t)((int64_t)stratum[r] - lo)]++] = KI{0, r};
        } else {   // stable radix sort on the label's order-preserving image
            for (int64_t r = 0; r < n; ++r) a[r] = KI{(uint64_t)((uint32_t)stratum[r] ^ 0x80000000u), r};
            radix_by_key(a.data(), tmp.data(), n);
            for (int64_t r = 0; r < n; ++r)
                if (r == 0 || a[r].k != a[r - 1].k) seg.push_back(r);
        }
        seg.push_back(n);
    }
    // 2. inside each stratum: time descending, original index ascending
    for (size_t g = 0; g + 1 < seg.size(); ++g) {
        KI *b = a.data() + seg[g];
        const int64_t len = seg[g + 1] - seg[g];
        for (int64_t r = 0; r < len; ++r) b[r].k = desc_key(time[b[r].i]);
        sort_by_key(b, tmp.data(), len);
    }
    // 3. row words
    perm.resize((size_t)n);
    meta.assign((size_t)n, 0u);
    for (size_t g = 0; g + 1 < seg.size(); ++g) {
        uint32_t gcount = 0;
        for (int64_t r = seg[g]; r < seg[g + 1]; ++r) {
            perm[r] = a[r].i;
            if (r == seg[g]) meta[r] |= kHeadBit;
            else if (a[r].k != a[r - 1].k) gcount = 0;
            if (event[a[r].i]) {
                meta[r] |= kEventBit;
                ++gcount;
            }
            if (r + 1 == seg[g + 1] || a[r + 1].k != a[r].k) meta[r] |= gcount;
        }
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
