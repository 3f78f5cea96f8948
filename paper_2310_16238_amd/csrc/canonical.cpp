// canonical.cpp -- see canonical.h.
#include "canonical.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

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

// Stable LSD radix sort of a[0, n) by bits 32..63 (8-bit digits; a digit on which every
// element agrees is skipped); the low 32 bits ride along.  All digit histograms are taken in
// one read pass.  tmp: scratch of n elements.
void radix_hi32(uint64_t *a, uint64_t *tmp, int64_t n)
{
    std::vector<uint32_t> hist(4 * 256, 0u);
    for (int64_t r = 0; r < n; ++r) {
        const uint64_t v = a[r] >> 32;
        ++hist[0 * 256 + (v & 0xff)];
        ++hist[1 * 256 + ((v >> 8) & 0xff)];
        ++hist[2 * 256 + ((v >> 16) & 0xff)];
        ++hist[3 * 256 + ((v >> 24) & 0xff)];
    }
    uint64_t *src = a, *dst = tmp;
    for (int d = 0; d < 4; ++d) {
        const uint32_t *h = &hist[(size_t)d * 256];
        bool trivial = false;
        for (int v = 0; v < 256; ++v) trivial |= (int64_t)h[v] == n;
        if (trivial) continue;
        uint32_t off[256];
        uint32_t sum = 0;
        for (int v = 0; v < 256; ++v) {
            off[v] = sum;
            sum += h[v];
        }
        const int shift = 32 + 8 * d;
        for (int64_t r = 0; r < n; ++r) dst[off[(src[r] >> shift) & 0xff]++] = src[r];
        std::swap(src, dst);
    }
    if (src != a) std::memcpy(a, src, sizeof(uint64_t) * (size_t)n);
}

}  // namespace

void canonical_order(int64_t n, const double *time, const uint8_t *event, const int32_t *stratum,
                     std::vector<int64_t> &perm, std::vector<uint32_t> &meta)
{
    // 1. every row by time descending, then original index ascending: an LSD radix sort of
    //    (top 32 bits of the order-preserving time key, row index) words, then each run of equal
    //    top bits put in full-key order by a stable sort (equal times keep the index order).
    //    Row indices fit in 32 bits (n <= 2^29 - 1).
    std::unique_ptr<uint64_t[]> key(new uint64_t[(size_t)n]), a(new uint64_t[(size_t)n]),
        tmp(new uint64_t[(size_t)n]);   // every entry is written before it is read
    for (int64_t r = 0; r < n; ++r) {
        key[(size_t)r] = desc_key(time[r]);
        a[(size_t)r] = (key[(size_t)r] & 0xffffffff00000000ull) | (uint64_t)r;
    }
    radix_hi32(a.get(), tmp.get(), n);
    const uint64_t *kp = key.get();
    auto full_less = [kp](uint64_t x, uint64_t y) { return kp[x & 0xffffffffu] < kp[y & 0xffffffffu]; };
    for (int64_t s0 = 0; s0 < n;) {
        int64_t s1 = s0 + 1;
        while (s1 < n && (a[(size_t)s1] >> 32) == (a[(size_t)s0] >> 32)) ++s1;
        if (s1 - s0 > 1) {
            uint64_t *b = a.get() + s0;
            const int64_t len = s1 - s0;
            if (len <= 32) {   // insertion sort (stable)
                for (int64_t r = 1; r < len; ++r) {
                    const uint64_t v = b[r];
                    int64_t q = r - 1;
                    while (q >= 0 && full_less(v, b[q])) {
                        b[q + 1] = b[q];
                        --q;
                    }
                    b[q + 1] = v;
                }
            } else {
                std::stable_sort(b, b + len, full_less);
            }
        }
        s0 = s1;
    }
    // 2. grouped by stratum (ascending label), the order of step 1 kept inside a stratum; the
    //    time key travels with each row for the tie-group test of step 3
    perm.resize((size_t)n);                  // row index of each canonical position
    int64_t *order = perm.data();
    uint64_t *okey = tmp.get();              // its time key
    std::vector<int64_t> seg;                // start of each stratum's run, then n
    if (!stratum) {
        for (int64_t r = 0; r < n; ++r) {
            order[r] = (int64_t)(a[(size_t)r] & 0xffffffffu);
            okey[r] = kp[order[r]];
        }
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
                if (start[(size_t)c + 1] > 0) seg.push_back(start[(size_t)c]);   // a label that occurs
                start[(size_t)c + 1] += start[(size_t)c];
            }
            for (int64_t q = 0; q < n; ++q) {
                const int64_t r = (int64_t)(a[(size_t)q] & 0xffffffffu);
                const int64_t at = start[(size_t)((int64_t)stratum[r] - lo)]++;
                order[at] = r;
                okey[at] = kp[r];
            }
        } else {   // stable radix sort on the label's order-preserving image, positions of step 1 riding along
            std::vector<uint64_t> lab((size_t)n), scratch((size_t)n);
            for (int64_t q = 0; q < n; ++q) {
                const int64_t r = (int64_t)(a[(size_t)q] & 0xffffffffu);
                lab[(size_t)q] = ((uint64_t)((uint32_t)stratum[r] ^ 0x80000000u) << 32) | (uint64_t)q;
            }
            radix_hi32(lab.data(), scratch.data(), n);
            for (int64_t q = 0; q < n; ++q) {
                order[q] = (int64_t)(a[(size_t)(lab[(size_t)q] & 0xffffffffu)] & 0xffffffffu);
                okey[q] = kp[order[q]];
                if (q == 0 || (lab[(size_t)q] >> 32) != (lab[(size_t)q - 1] >> 32)) seg.push_back(q);
            }
        }
        seg.push_back(n);
    }
    // 3. row words
    meta.assign((size_t)n, 0u);
    for (size_t g = 0; g + 1 < seg.size(); ++g) {
        uint32_t gcount = 0;
        for (int64_t r = seg[g]; r < seg[g + 1]; ++r) {
            if (r == seg[g]) meta[(size_t)r] |= kHeadBit;
            else if (okey[r] != okey[r - 1]) gcount = 0;
            if (event[order[r]]) {
                meta[(size_t)r] |= kEventBit;
                ++gcount;
            }
            if (r + 1 == seg[g + 1] || okey[r + 1] != okey[r]) meta[(size_t)r] |= gcount;
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
