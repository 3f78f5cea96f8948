// Host-only program for the sanitizer test: exercises the library's host code
// (input checks, canonical order, interval split) on random and edge-case
// inputs, checking the canonical order against a plain sort.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers_cpu.py.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "canonical.h"
#include "coxmi.h"

static int fails = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++fails;                                                    \
        }                                                               \
    } while (0)

static void one_case(std::mt19937_64 &g, int64_t n, int nstrata, int ties, int p)
{
    std::vector<double> time(n), x((size_t)(n * p));
    std::vector<uint8_t> event(n);
    std::vector<int32_t> stratum(n);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    for (int64_t i = 0; i < n; ++i) {
        time[i] = ties ? std::floor(u(g) * ties) : u(g);
        if (u(g) < 0.1) time[i] = -0.0;
        event[i] = u(g) < 0.5;
        stratum[i] = (int32_t)(g() % (uint64_t)nstrata) * 3 - 7;
    }
    for (auto &v : x) v = u(g) - 0.5;
    std::vector<int64_t> perm;
    std::vector<uint32_t> meta;
    CHECK(coxmi::check_data(n, p, n, x.data(), time.data(), event.data()) == nullptr);
    coxmi::canonical_order(n, time.data(), event.data(), stratum.data(), perm, meta);
    CHECK((int64_t)perm.size() == n && (int64_t)meta.size() == n);
    // reference: sort by (stratum asc, time desc with -0 == +0, index asc)
    std::vector<int64_t> ref(n);
    for (int64_t i = 0; i < n; ++i) ref[i] = i;
    std::sort(ref.begin(), ref.end(), [&](int64_t a, int64_t b) {
        if (stratum[a] != stratum[b]) return stratum[a] < stratum[b];
        const double ta = time[a] + 0.0, tb = time[b] + 0.0;
        if (ta != tb) return ta > tb;
        return a < b;
    });
    CHECK(perm == ref);
    int64_t events = 0, dsum = 0;
    for (int64_t c = 0; c < n; ++c) {
        events += event[perm[c]];
        dsum += meta[c] & 0x1fffffffu;
        const bool head = c == 0 || stratum[perm[c]] != stratum[perm[c - 1]];
        CHECK(((meta[c] >> 31) & 1u) == (head ? 1u : 0u));
    }
    CHECK(events == dsum);
    // interval split with a few cuts and step coefficients
    cox_data d{};
    d.n = n;
    d.p = p;
    d.x = x.data();
    d.ldx = n;
    d.time = time.data();
    d.event = event.data();
    d.stratum = stratum.data();
    std::vector<double> cuts = {0.2, 0.5, 0.9};
    if (ties) cuts = {1.0, (double)(ties / 2)};
    std::vector<uint8_t> tv(p, 0);
    tv[0] = 1;
    cox_intervals *s = nullptr;
    CHECK(cox_split_intervals(&d, (int)cuts.size(), cuts.data(), tv.data(), nullptr, &s) == COX_OK);
    if (s) {
        int64_t ev = 0;
        for (int64_t r = 0; r < s->data.n; ++r) ev += s->data.event[r];
        CHECK(ev == events);
        CHECK(s->data.p == p + (int64_t)cuts.size());
        cox_intervals_release(s);
    }
}

int main()
{
    std::mt19937_64 g(12345);
    const int64_t sizes[] = {1, 2, 3, 17, 256, 4095, 4096, 4097, 20000};
    for (int64_t n : sizes)
        for (int ns : {1, 3, 50})
            for (int ties : {0, 7})
                one_case(g, n, ns, ties, 3);
    // error paths must not touch memory they should not
    std::vector<double> t = {1.0, std::nan("")};
    std::vector<uint8_t> e = {1, 2};
    double x2[2] = {0.0, 0.0};
    CHECK(coxmi::check_data(2, 1, 2, x2, t.data(), e.data()) != nullptr);
    CHECK(coxmi::check_data(0, 1, 2, x2, t.data(), e.data()) != nullptr);
    double xx[2] = {1.0, 2.0}, tt[2] = {1.0, 2.0}, bad_cuts[2] = {2.0, 1.0};
    uint8_t ee[2] = {1, 0};
    cox_data d{};
    d.n = 2;
    d.p = 1;
    d.x = xx;
    d.ldx = 2;
    d.time = tt;
    d.event = ee;
    cox_intervals *s = nullptr;
    CHECK(cox_split_intervals(&d, 2, bad_cuts, nullptr, nullptr, &s) == COX_EINVAL && s == nullptr);
    CHECK(cox_split_intervals(&d, -1, nullptr, nullptr, nullptr, &s) == COX_EINVAL);
    cox_intervals_release(nullptr);
    std::printf(fails ? "FAILED %d\n" : "OK\n", fails);
    return fails ? 1 : 0;
}
