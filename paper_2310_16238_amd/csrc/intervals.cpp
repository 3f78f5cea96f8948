// intervals.cpp -- the interval-stratified augmented data set of Secs. 2.2-2.3
// (host, integer bookkeeping and copies; the fit itself is the ordinary
// stratified path).  See cox_split_intervals in coxmi.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <type_traits>
#include <vector>

#include "canonical.h"
#include "coxmi.h"

namespace {

struct Store {
    std::vector<double> x, time;
    std::vector<uint8_t> event;
    std::vector<int32_t> stratum;
    std::vector<int64_t> row_subject;
    std::vector<int32_t> row_interval, col_source, col_interval;
};

// Standard layout with the public part first, so a cox_intervals pointer handed
// out converts back to its Intervals.
struct Intervals {
    cox_intervals pub;
    Store *store;
};
static_assert(std::is_standard_layout<Intervals>::value, "the public part converts back to its owner");

}  // namespace

extern "C" int cox_split_intervals(const cox_data *d, int ncuts, const double *cuts, const uint8_t *tv_coef,
                                   const double *x_by_interval, cox_intervals **out)
{
    if (!out) return COX_EINVAL;
    *out = nullptr;
    if (!d) return COX_EINVAL;
    if (coxmi::check_data(d->n, d->p, d->ldx, d->x, d->time, d->event)) return COX_EINVAL;
    if (ncuts < 0 || (ncuts > 0 && !cuts)) return COX_EINVAL;
    for (int k = 0; k < ncuts; ++k) {
        if (!std::isfinite(cuts[k])) return COX_EINVAL;
        if (k > 0 && !(cuts[k] > cuts[k - 1])) return COX_EINVAL;
    }
    const int64_t n = d->n, p = d->p;
    const int K = ncuts + 1;
    // interval k = [lo_k, hi_k): lo_0 = -inf, hi_{K-1} = +inf
    auto lo = [&](int k) { return k == 0 ? -std::numeric_limits<double>::infinity() : cuts[k - 1]; };
    auto hi = [&](int k) { return k == K - 1 ? std::numeric_limits<double>::infinity() : cuts[k]; };

    // rank of each subject's stratum label among the distinct labels
    std::vector<int32_t> srank((size_t)n, 0);
    int64_t nstrata = 1;
    if (d->stratum) {
        std::vector<int32_t> labels(d->stratum, d->stratum + n);
        std::sort(labels.begin(), labels.end());
        labels.erase(std::unique(labels.begin(), labels.end()), labels.end());
        nstrata = (int64_t)labels.size();
        for (int64_t i = 0; i < n; ++i)
            srank[i] = (int32_t)(std::lower_bound(labels.begin(), labels.end(), d->stratum[i]) - labels.begin());
    }
    if (nstrata * K > (int64_t)std::numeric_limits<int32_t>::max()) return COX_EINVAL;

    // augmented rows
    int64_t naug = 0;
    for (int k = 0; k < K; ++k)
        for (int64_t i = 0; i < n; ++i) naug += d->time[i] >= lo(k) ? 1 : 0;
    if (naug > (int64_t)std::numeric_limits<int32_t>::max()) return COX_EINVAL;

    Intervals *owner = new (std::nothrow) Intervals();
    Store *r = owner ? new (std::nothrow) Store() : nullptr;
    if (!r) {
        delete owner;
        return COX_ENOMEM;
    }
    owner->store = r;
    cox_intervals &pub = owner->pub;
    try {
        // augmented columns
        for (int64_t j = 0; j < p; ++j) {
            if (tv_coef && tv_coef[j]) {
                for (int k = 0; k < K; ++k) {
                    r->col_source.push_back((int32_t)j);
                    r->col_interval.push_back(k);
                }
            } else {
                r->col_source.push_back((int32_t)j);
                r->col_interval.push_back(-1);
            }
        }
        const int64_t paug = (int64_t)r->col_source.size();
        r->time.resize((size_t)naug);
        r->event.resize((size_t)naug);
        r->stratum.resize((size_t)naug);
        r->row_subject.resize((size_t)naug);
        r->row_interval.resize((size_t)naug);
        int64_t a = 0;
        for (int k = 0; k < K; ++k)
            for (int64_t i = 0; i < n; ++i) {
                const double y = d->time[i];
                if (!(y >= lo(k))) continue;
                const bool inside = y < hi(k);
                r->time[a] = inside ? y : hi(k);
                r->event[a] = inside ? d->event[i] : 0;
                r->stratum[a] = (int32_t)(srank[i] * (int64_t)K + k);
                r->row_subject[a] = i;
                r->row_interval[a] = k;
                ++a;
            }
        r->x.assign((size_t)(naug * paug), 0.0);
        for (int64_t c = 0; c < paug; ++c) {
            const int64_t j = r->col_source[c];
            const int kc = r->col_interval[c];
            double *col = r->x.data() + c * naug;
            for (int64_t b = 0; b < naug; ++b) {
                const int k = r->row_interval[b];
                if (kc >= 0 && kc != k) continue;   // a step coefficient's column is zero off its interval
                const int64_t i = r->row_subject[b];
                const double *src = x_by_interval ? x_by_interval + (int64_t)k * d->ldx * p : d->x;
                col[b] = src[j * d->ldx + i];
            }
        }
        pub.data.n = naug;
        pub.data.p = paug;
        pub.data.x = r->x.data();
        pub.data.ldx = naug;
        pub.data.time = r->time.data();
        pub.data.event = r->event.data();
        pub.data.stratum = r->stratum.data();
        pub.intervals = K;
        pub.row_subject = r->row_subject.data();
        pub.row_interval = r->row_interval.data();
        pub.col_source = r->col_source.data();
        pub.col_interval = r->col_interval.data();
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
