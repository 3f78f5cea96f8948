// resample.h -- launchers of resample.hip for indicator X (dense X: internal.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace coxmi {

// Child unit u of column j takes bit i from parent row src[u * ipt_out + i] (-1: 0) of parent
// column col_src[j] (NULL: j); with rint and col_int, a column with col_int[j] >= 0 keeps only
// rows whose rint equals it.  Units are uint8 (ipt <= 8) or uint16 (ipt 16) on both sides.
// Returns a hipError_t value.
int launch_gather_bits(const void *b_in, int64_t ldb_in, int ipt_in, const int32_t *src, const int32_t *rint,
                       const int32_t *col_src, const int32_t *col_int, void *b_out, int64_t ldb_out, int ipt_out, int p,
                       hipStream_t stream);

// q[j] for indicator X: the number of event rows whose bit is set (fixed-order sums).
int launch_event_sums_bits(const void *bits, int64_t ldb, int ipt, const uint32_t *meta, double *q, int p,
                           hipStream_t stream);

}  // namespace coxmi
