// intervals.cpp -- the interval-stratified augmented data set of Secs. 2.2-2.3
// (host, integer bookkeeping and copies; the fit itself is the ordinary
// stratified path).  See cox_split_intervals in coxmi.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <new>
#include <system_error>
#include <thread>
#include <type_traits>
#include <vector>

#include "canonical.h"
#include "coxmi.h"
#include "intervals.h"

namespace {

struct Store {
    std::unique_ptr<double[]> x;    // not zero-filled: every entry is written by the column fill
    coxmi::IntervalRows rows;
};

// Standard layout with the public part first, so a cox_intervals pointer handed
// out converts back to its Intervals.
struct Intervals {
    cox_intervals pub;
    Store *store;
};
static_assert(std::is_standard_layout<Intervals>::value, "the public part converts back to its owner");

}  // namespace

namespace coxmi {

int interval_rows(int64_t n, const double *time, const uint8_t *event, const int32_t *stratum, int ncuts,
                  const double *cuts, const uint8_t *tv_coef, int64_t p, IntervalRows &r)
{
    if (ncuts < 0 || (ncuts > 0 && !cuts)) return COX_EINVAL;
    for (int k = 0; k < ncuts; ++k) {
        if (!std::isfinite(cuts[k])) return COX_EINVAL;
        if (k > 0 && !(cuts[k] > cuts[k - 1])) return COX_EINVAL;
    }
    const int K = ncuts + 1;
    // interval k = [lo_k, hi_k): lo_0 = -inf, hi_{K-1} = +inf
    auto lo = [&](int k) { return k == 0 ? -std::numeric_limits<double>::infinity() : cuts[k - 1]; };
    auto hi = [&](int k) { return k == K - 1 ? std::numeric_limits<double>::infinity() : cuts[k]; };

    // rank of each subject's stratum label among the distinct labels
    std::vector<int32_t> srank((size_t)n, 0);
    int64_t nstrata = 1;
    if (stratum) {
        std::vector<int32_t> labels(stratum, stratum + n);
        std::sort(labels.begin(), labels.end());
        labels.erase(std::unique(labels.begin(), labels.end()), labels.end());
        nstrata = (int64_t)labels.size();
        for (int64_t i = 0; i < n; ++i)
            srank[i] = (int32_t)(std::lower_bound(labels.begin(), labels.end(), stratum[i]) - labels.begin());
    }
    if (nstrata * K > (int64_t)std::numeric_limits<int32_t>::max()) return COX_EINVAL;

    int64_t naug = 0;
    for (int k = 0; k < K; ++k)
        for (int64_t i = 0; i < n; ++i) naug += time[i] >= lo(k) ? 1 : 0;
    if (naug > (int64_t)std::numeric_limits<int32_t>::max()) return COX_EINVAL;

    r.intervals = K;
    r.col_source.clear();
    r.col_interval.clear();
    for (int64_t j = 0; j < p; ++j) {
        if (tv_coef && tv_coef[j]) {
            for (int k = 0; k < K; ++k) {
                r.col_source.push_back((int32_t)j);
                r.col_interval.push_back(k);
            }
        } else {
            r.col_source.push_back((int32_t)j);
            r.col_interval.push_back(-1);
        }
    }
    r.time.resize((size_t)naug);
    r.event.resize((size_t)naug);
    r.stratum.resize((size_t)naug);
    r.row_subject.resize((size_t)naug);
    r.row_interval.resize((size_t)naug);
    int64_t a = 0;
    for (int k = 0; k < K; ++k)
        for (int64_t i = 0; i < n; ++i) {
            const double y = time[i];
            if (!(y >= lo(k))) continue;
            const bool inside = y < hi(k);
            r.time[(size_t)a] = inside ? y : hi(k);
            r.event[(size_t)a] = inside ? event[i] : 0;
            r.stratum[(size_t)a] = (int32_t)(srank[(size_t)i] * (int64_t)K + k);
            r.row_subject[(size_t)a] = i;
            r.row_interval[(size_t)a] = k;
            ++a;
        }
    return COX_OK;
}

}  // namespace coxmi

extern "C" int cox_split_intervals(const cox_data *d, int ncuts, const double *cuts, const uint8_t *tv_coef,
                                   const double *x_by_interval, cox_intervals **out)
{
    if (!out) return COX_EINVAL;
    *out = nullptr;
    if (!d) return COX_EINVAL;
    if (coxmi::check_data(d->n, d->p, d->ldx, d->x, d->time, d->event)) return COX_EINVAL;
    const int64_t n = d->n, p = d->p;
    Intervals *owner = new (std::nothrow) Intervals();
    Store *r = owner ? new (std::nothrow) Store() : nullptr;
    if (!r) {
        delete owner;
        return COX_ENOMEM;
    }
    owner->store = r;
    cox_intervals &pub = owner->pub;
    try {
        const int rc = coxmi::interval_rows(n, d->time, d->event, d->stratum, ncuts, cuts, tv_coef, p, r->rows);
        if (rc != COX_OK) {
            delete r;
            delete owner;
            return rc;
        }
        const int K = r->rows.intervals;
        const int64_t naug = (int64_t)r->rows.time.size();
        const int64_t paug = (int64_t)r->rows.col_source.size();
        // interval k's rows are the contiguous block [first[k], first[k + 1])
        std::vector<int64_t> first((size_t)K + 1, 0);
        for (int64_t b = 0; b < naug; ++b) first[(size_t)r->rows.row_interval[b] + 1]++;
        for (int k = 0; k < K; ++k) first[(size_t)k + 1] += first[(size_t)k];
        r->x.reset(new double[(size_t)(naug * paug)]);
        // columns are independent: fill them on a few threads (each column a gather per interval)
        auto fill = [&](int64_t c0, int64_t c1) {
            for (int64_t c = c0; c < c1; ++c) {
                const int64_t j = r->rows.col_source[(size_t)c];
                const int kc = r->rows.col_interval[(size_t)c];
                double *col = r->x.get() + c * naug;
                for (int k = 0; k < K; ++k) {
                    double *dst = col + first[(size_t)k];
                    const int64_t len = first[(size_t)k + 1] - first[(size_t)k];
                    if (kc >= 0 && kc != k) {   // a step coefficient's column is zero off its interval
                        std::fill(dst, dst + len, 0.0);
                        continue;
                    }
                    const double *src = (x_by_interval ? x_by_interval + (int64_t)k * d->ldx * p : d->x) + j * d->ldx;
                    const int64_t *subj = r->rows.row_subject.data() + first[(size_t)k];
                    for (int64_t b = 0; b < len; ++b) dst[b] = src[subj[b]];
                }
            }
        };
        const int64_t work = naug * paug;
        int nth = (int)std::min<int64_t>(std::max(1u, std::thread::hardware_concurrency()), 16);
        nth = (int)std::min<int64_t>(nth, std::max<int64_t>(1, work >> 22));
        nth = (int)std::min<int64_t>(nth, paug);
        if (nth <= 1) {
            fill(0, paug);
        } else {
            std::vector<std::thread> pool;
            const int64_t per = (paug + nth - 1) / nth;
            for (int t = 0; t < nth; ++t) {
                const int64_t c0 = t * per, c1 = std::min<int64_t>(paug, c0 + per);
                if (c0 >= c1) continue;
                try {
                    pool.emplace_back(fill, c0, c1);
                } catch (const std::system_error &) {   // no thread to spare: fill this block here
                    fill(c0, c1);
                }
            }
            for (auto &th : pool) th.join();
        }
        pub.data.n = naug;
        pub.data.p = paug;
        pub.data.x = r->x.get();
        pub.data.ldx = naug;
        pub.data.time = r->rows.time.data();
        pub.data.event = r->rows.event.data();
        pub.data.stratum = r->rows.stratum.data();
        pub.intervals = K;
        pub.row_subject = r->rows.row_subject.data();
        pub.row_interval = r->rows.row_interval.data();
        pub.col_source = r->rows.col_source.data();
        pub.col_interval = r->rows.col_interval.data();
    } catch (const std::bad_alloc &) {
        delete r;
        delete owner;
        return COX_ENOMEM;
    }
    *out = &pub;
    return COX_OK;
}

extern "C" void cox_intervals_release(cox_intervals *s)
{
    if (!s) return;
    Intervals *owner = reinterpret_cast<Intervals *>(s);   // pub is its first member
    delete owner->store;
    delete owner;
}
