// canonical.h -- the canonical row order of a data set (host, integer work).
//
// Rows are sorted by stratum ascending, time descending and original index
// ascending (Sec. 2.7: strata concatenated, each in decreasing time), and
// every row gets a 32-bit word: bit 31 marks the first row of a stratum,
// bit 30 an event, and the last row of each tie group carries the number of
// events of the group in bits 0..28 (ties: every row with an equal or later
// time is at risk, so all events of a group read the risk-set sums at its
// last row).
#pragma once

#include <stdint.h>

#include <vector>

namespace coxmi {

// perm[i] = original index of canonical row i; meta[i] = its row word.
// stratum may be NULL (one stratum).  Inputs must already be validated.
void canonical_order(int64_t n, const double *time, const uint8_t *event, const int32_t *stratum,
                     std::vector<int64_t> &perm, std::vector<uint32_t> &meta);

// Checks shared by every entry point that takes a data set: returns nullptr
// when (n, p, ldx, x, time, event) are usable, else a message.
const char *check_data(int64_t n, int64_t p, int64_t ldx, const double *x, const double *time,
                       const uint8_t *event);

}  // namespace coxmi
