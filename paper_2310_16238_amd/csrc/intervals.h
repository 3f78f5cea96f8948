// intervals.h -- rows and columns of the interval-stratified data set of
// Secs. 2.2-2.3, shared by cox_split_intervals (host copy of the augmented X)
// and cox_init_intervals (augmented X gathered on the device).
#pragma once

#include <stdint.h>

#include <vector>

namespace coxmi {

struct IntervalRows {
    int intervals = 1;
    std::vector<double> time;              // min(Y_i, t_k)
    std::vector<uint8_t> event;            // delta_i if Y_i lies in interval k
    std::vector<int32_t> stratum;          // rank(s_i) * K + k
    std::vector<int64_t> row_subject;      // i
    std::vector<int32_t> row_interval;     // k
    std::vector<int32_t> col_source, col_interval;   // columns: source column, interval or -1
};

// Interval-major rows (k, i) for every i with Y_i >= t_{k-1}, subjects in order, and the
// augmented columns (a step-coefficient column j becomes K columns).  Returns COX_OK or
// COX_EINVAL (bad cuts, too many rows or strata); may throw std::bad_alloc.
int interval_rows(int64_t n, const double *time, const uint8_t *event, const int32_t *stratum, int ncuts,
                  const double *cuts, const uint8_t *tv_coef, int64_t p, IntervalRows &r);

}  // namespace coxmi
