// coxmi.cpp -- C ABI of the stratified Cox library (declared in include/coxmi.h).
//
// Host-side work is limited to what is done once per data set: input checks,
// the canonical row order of Sec. 2.7 (integer work, exact), tie groups, and
// copying X into device memory in that order.  Everything per iteration runs
// in the persistent kernel (ccd_kernel.hip).
#include "coxmi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "canonical.h"
#include "handle.h"
#include "internal.h"
#include "intervals.h"
#include "newton.h"
#include "resample.h"

using namespace coxmi;

static thread_local std::string g_init_error;

static int fail(cox_handle *h, int code, const std::string &msg)
{
    if (h) h->err = msg;
    else g_init_error = msg;
    return code;
}

static int hip_fail(cox_handle *h, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(h, e == hipErrorOutOfMemory ? COX_ENOMEM : COX_EDEVICE, m);
}

int handle_fail(cox_handle *h, int code, const std::string &msg) { return fail(h, code, msg); }
int handle_hip_fail(cox_handle *h, hipError_t e, const char *what) { return hip_fail(h, e, what); }

extern "C" void cox_default_options(cox_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->gamma = 0.0;
    o->penalize = nullptr;
    o->mode = COX_CCD;
    o->x_precision = COX_F64;
    o->ties = COX_BRESLOW;
    o->tol = 1e-12;
    o->max_iter = 1000;
    o->stream = nullptr;
}

static void free_device(cox_handle *h)
{
    newton_free(h);
    if (h->d_x) (void)hipFree(h->d_x);
    if (h->d_xbits) (void)hipFree(h->d_xbits);
    if (h->d_xvals) (void)hipFree(h->d_xvals);
    if (h->d_xvoff) (void)hipFree(h->d_xvoff);
    if (h->d_woff) (void)hipFree(h->d_woff);
    if (h->d_trust) (void)hipFree(h->d_trust);
    h->d_xbits = nullptr;
    h->d_xvals = nullptr;
    h->d_xvoff = nullptr;
    h->d_woff = nullptr;
    h->d_trust = nullptr;
    if (h->d_meta) (void)hipFree(h->d_meta);
    if (h->d_vec) (void)hipFree(h->d_vec);
    if (h->d_sync) (void)hipFree(h->d_sync);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    h->d_x = nullptr;
    h->d_meta = nullptr;
    h->d_vec = nullptr;
    h->d_sync = nullptr;
    h->ev0 = h->ev1 = nullptr;
}

// Device row of every canonical row when tiles hold R rows and no stratum that
// fits in one tile may cross a tile boundary (the gap is filled with padding
// rows).  Returns the padded length.
static int64_t aligned_positions(const std::vector<uint32_t> &meta, int64_t R, std::vector<int64_t> *pos)
{
    const int64_t n = (int64_t)meta.size();
    int64_t cur = 0, i = 0;
    while (i < n) {
        int64_t e = i + 1;
        while (e < n && !(meta[e] & kHeadBit)) ++e;
        const int64_t m = e - i;
        const int64_t room = R - (cur % R);
        if (m <= R && m > room) cur += room;
        if (pos)
            for (int64_t k = 0; k < m; ++k) (*pos)[i + k] = cur + k;
        cur += m;
        i = e;
    }
    return cur;
}

// Rows per thread, workgroups and device row positions for the persistent
// kernel: the fewest rows per thread whose workgroup count fits one per
// compute unit, preferring a layout in which no stratum crosses a wave's rows
// (then every wave's scan is its own, with no carry between waves), then one in
// which no stratum that fits a workgroup tile crosses a tile boundary.
static int choose_layout(const std::vector<uint32_t> &meta, int p, LaunchShape &shape,
                         std::vector<int64_t> &pos, std::string &err)
{
    const int64_t n = (int64_t)meta.size();
    pos.assign(n, 0);
    shape.wave = false;
    int64_t longest = 0;   // the longest stratum
    for (int64_t i = 0; i < n;) {
        int64_t e = i + 1;
        while (e < n && !(meta[e] & kHeadBit)) ++e;
        longest = std::max(longest, e - i);
        i = e;
    }
    const int ipts[] = {1, 2, 4, 8, 16};
    for (int ipt : ipts) {
        int groups = 0;
        if (max_resident_groups(ipt, p, &groups, err) != 0) return COX_EDEVICE;
        if (groups < 1) continue;
        const int64_t R = (int64_t)kThreads * ipt, Rw = (int64_t)kWaveRows * ipt;
        if (longest <= Rw) {
            const int64_t lw = aligned_positions(meta, Rw, nullptr);
            if ((lw + R - 1) / R <= groups) {
                aligned_positions(meta, Rw, &pos);
                shape.ipt = ipt;
                shape.grid = (int)((lw + R - 1) / R);
                shape.ld = (int64_t)shape.grid * R;
                shape.wave = true;
                return 0;
            }
        }
        const int64_t la = aligned_positions(meta, R, nullptr);
        if ((la + R - 1) / R <= groups) {
            aligned_positions(meta, R, &pos);
            shape.ipt = ipt;
            shape.grid = (int)((la + R - 1) / R);
            shape.ld = (int64_t)shape.grid * R;
            return 0;
        }
        if ((n + R - 1) / R <= groups) {
            std::iota(pos.begin(), pos.end(), int64_t(0));
            shape.ipt = ipt;
            shape.grid = (int)((n + R - 1) / R);
            shape.ld = (int64_t)shape.grid * R;
            return 0;
        }
    }
    err = "n exceeds the register-resident capacity of the persistent kernel (CUs x 512 x 16 rows)";
    return COX_EUNSUPPORTED;
}

// Layout for data sets beyond the persistent kernel (Newton fits only): tiles
// of kNewtonTile rows, stratum-aligned like the persistent layout.  ipt = 0
// marks that the persistent kernel cannot run on it.
constexpr int64_t kNewtonTile = 4096;

static void tile_layout(const std::vector<uint32_t> &meta, LaunchShape &shape, std::vector<int64_t> &pos)
{
    const int64_t n = (int64_t)meta.size();
    pos.assign(n, 0);
    const int64_t la = aligned_positions(meta, kNewtonTile, nullptr);
    if (la <= n + n / 8) {
        aligned_positions(meta, kNewtonTile, &pos);
    } else {
        std::iota(pos.begin(), pos.end(), int64_t(0));
    }
    const int64_t rows = la <= n + n / 8 ? la : n;
    shape.ipt = 0;
    shape.wave = false;
    shape.grid = (int)((rows + kNewtonTile - 1) / kNewtonTile);
    shape.ld = (int64_t)shape.grid * kNewtonTile;
}

// Bytes of one thread's unit of an indicator column (ipt bits).
static size_t indicator_unit(int ipt) { return ipt > 8 ? 2 : 1; }

// Device buffers of a handle whose layout (shape, pos) is set; dense X unless ldb != 0.
static hipError_t alloc_device(cox_handle *h)
{
    const int64_t ld = h->shape.ld, p = h->p;
    hipError_t e;
    if ((h->ldb == 0 && (e = hipMalloc(&h->d_x, sizeof(double) * (size_t)ld * p)) != hipSuccess) ||
        (h->ldb != 0 && (e = hipMalloc(&h->d_xbits, indicator_unit(h->shape.ipt) * (size_t)h->ldb * p)) != hipSuccess) ||
        (e = hipMalloc(&h->d_meta, sizeof(uint32_t) * (size_t)ld)) != hipSuccess ||
        (e = hipMalloc(&h->d_vec, sizeof(double) * (size_t)(6 * p + kResultSlots + 64))) != hipSuccess ||
        (e = hipMalloc(&h->d_sync, sync_scratch_bytes(h->shape.ipt ? h->shape.grid : 1))) != hipSuccess ||
        (h->shape.ipt && (e = hipMalloc(&h->d_trust, sizeof(double) * (size_t)h->shape.grid * p)) != hipSuccess))
        return e;
    return hipSuccess;
}

// Row words at the layout positions; padding rows are single-row strata without events.
static hipError_t upload_meta(cox_handle *h)
{
    const int64_t ld = h->shape.ld;
    std::vector<uint32_t> mpad(ld, kHeadBit | kPadBit);
    for (int64_t i = 0; i < h->n; ++i) mpad[h->pos[i]] = h->meta[i];
    return hipMemcpy(h->d_meta, mpad.data(), sizeof(uint32_t) * ld, hipMemcpyHostToDevice);
}

// l1 weights, the exponential's table and the timing events.
static hipError_t upload_tables(cox_handle *h)
{
    hipError_t e = hipMemcpy(h->gam(), h->gamma.data(), sizeof(double) * h->p, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        // 2^(j/64), j = 0..63, rounded to nearest from extended precision (table of the device exp)
        double tab[64];
        for (int j = 0; j < 64; ++j) tab[j] = (double)std::exp2l((long double)j / 64.0L);
        e = hipMemcpy(h->exp_tab(), tab, sizeof(tab), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipEventCreate(&h->ev0);
    if (e == hipSuccess) e = hipEventCreate(&h->ev1);
    return e;
}

// Options common to cox_init and cox_init_resample; 0 or a COX_* code with msg set.
static int check_options(const cox_options &opt, std::string &msg)
{
    if (opt.mode != COX_CCD && opt.mode != COX_NEWTON_REFINE) { msg = "unknown mode"; return COX_EINVAL; }
    if (opt.x_precision != COX_F64 && opt.x_precision != COX_BF16 && opt.x_precision != COX_FP8_E4M3) {
        msg = "x_precision must be COX_F64, COX_BF16 or COX_FP8_E4M3";
        return COX_EUNSUPPORTED;
    }
    if (opt.x_precision == COX_FP8_E4M3 && opt.mode != COX_NEWTON_REFINE) {
        msg = "COX_FP8_E4M3 applies to COX_NEWTON_REFINE fits";
        return COX_EUNSUPPORTED;
    }
    if (opt.ties != COX_BRESLOW && opt.ties != COX_EFRON) { msg = "ties must be COX_BRESLOW or COX_EFRON"; return COX_EINVAL; }
    if (!(opt.gamma >= 0.0) || !std::isfinite(opt.gamma)) { msg = "gamma must be finite and >= 0"; return COX_EINVAL; }
    if (!(opt.tol >= 0.0)) { msg = "tol must be >= 0"; return COX_EINVAL; }
    if (opt.max_iter < 1) { msg = "max_iter must be >= 1"; return COX_EINVAL; }
    return 0;
}

// Launch layout for h->meta (sets shape and pos); Newton fits fall back to the tile layout.
// dense: the handle will hold FP64 X, so the full evaluation and Newton fits can serve a COX_CCD
// handle too long for the persistent kernel (p <= kMaxNewtonP).
static int layout_for(cox_handle *h, std::string &err, bool dense)
{
    int rc = choose_layout(h->meta, (int)h->p, h->shape, h->pos, err);
    if (rc == COX_EUNSUPPORTED &&
        (h->opt.mode == COX_NEWTON_REFINE || (dense && h->p <= kMaxNewtonP))) {
        tile_layout(h->meta, h->shape, h->pos);
        rc = 0;
    }
    return rc;
}

bool coxmi::device_range_ok(const void *ptr, size_t bytes, int device)
{
    if (!ptr) return false;
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess ||
        (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged) || a.device != device) {
        (void)hipGetLastError();
        return false;
    }
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void *>(ptr)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const char *b = static_cast<const char *>(base), *q = static_cast<const char *>(ptr);
    if (q < b || (size_t)(q - b) > size) return false;
    return bytes <= size - (size_t)(q - b);
}

// Host copies of device-resident keys (time, event, stratum), read on `stream` after the
// work already queued there.  Returns nullptr or a message.
static const char *copy_keys(const cox_data *d, hipStream_t stream, std::vector<double> &time,
                             std::vector<uint8_t> &event, std::vector<int32_t> &stratum)
{
    const int64_t n = d->n, p = d->p;
    if (n < 1 || p < 1) return "need n >= 1 and p >= 1";
    if (d->ldx < n) return "ldx < n";
    if (!d->x || !d->time || !d->event) return "x, time and event are required";
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "cannot query the current device";
    const size_t xbytes = sizeof(double) * ((size_t)d->ldx * (size_t)(p - 1) + (size_t)n);
    if (!device_range_ok(d->x, xbytes, dev) || !device_range_ok(d->time, sizeof(double) * (size_t)n, dev) ||
        !device_range_ok(d->event, (size_t)n, dev) ||
        (d->stratum && !device_range_ok(d->stratum, sizeof(int32_t) * (size_t)n, dev)))
        return "on_device data must lie in device memory of the current device (x: ldx * (p - 1) + n doubles)";
    time.resize((size_t)n);
    event.resize((size_t)n);
    if (d->stratum) stratum.resize((size_t)n);
    hipError_t e = hipMemcpyAsync(time.data(), d->time, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(event.data(), d->event, (size_t)n, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess && d->stratum)
        e = hipMemcpyAsync(stratum.data(), d->stratum, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return "copying the device-resident keys failed";
    }
    return nullptr;
}

extern "C" int cox_init(cox_handle **out, const cox_data *d, const cox_options *o)
{
    if (!out) return fail(nullptr, COX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d) return fail(nullptr, COX_EINVAL, "data is NULL");
    const int64_t n = d->n, p = d->p;
    if (n > (int64_t)kCountMask) return fail(nullptr, COX_EUNSUPPORTED, "n exceeds 2^29 - 1");
    cox_options opt;
    if (o) opt = *o;
    else cox_default_options(&opt);
    {
        std::string msg;
        if (const int rc = check_options(opt, msg)) return fail(nullptr, rc, msg);
    }
    // the keys on the host: the caller's arrays, or copies of device-resident ones
    const double *time = d->time;
    const uint8_t *event = d->event;
    const int32_t *stratum = d->stratum;
    std::vector<double> time_h;
    std::vector<uint8_t> event_h;
    std::vector<int32_t> stratum_h;
    if (d->on_device) {
        if (const char *bad = copy_keys(d, static_cast<hipStream_t>(opt.stream), time_h, event_h, stratum_h))
            return fail(nullptr, COX_EINVAL, bad);
        time = time_h.data();
        event = event_h.data();
        stratum = d->stratum ? stratum_h.data() : nullptr;
    }
    if (const char *bad = check_data(n, p, d->ldx, d->x, time, event)) return fail(nullptr, COX_EINVAL, bad);
    if (p > kMaxCcdP || (opt.mode == COX_NEWTON_REFINE && p > kMaxNewtonP))
        return fail(nullptr, COX_EUNSUPPORTED, "p exceeds 12288 (COX_CCD) or 4096 (COX_NEWTON_REFINE)");
    if (opt.x_precision == COX_FP8_E4M3 && p > kMaxFp8P)
        return fail(nullptr, COX_EUNSUPPORTED, "the FP8 contraction supports p <= 4096");

    cox_handle *h = new cox_handle();
    h->n = n;
    h->p = p;
    h->opt = opt;
    h->opt.penalize = nullptr;
    h->stream = static_cast<hipStream_t>(opt.stream);
    (void)hipGetDevice(&h->device);

    // canonical order: stratum ascending, time descending, original index ascending
    canonical_order(n, time, event, stratum, h->perm, h->meta);

    h->gamma.assign(p, opt.gamma);
    if (o && o->penalize)
        for (int64_t j = 0; j < p; ++j) h->gamma[j] = o->penalize[j] ? opt.gamma : 0.0;

    std::string err;
    const int rc = layout_for(h, err, true);
    if (rc != 0) {
        delete h;
        return fail(nullptr, rc, err);
    }
    const int64_t ld = h->shape.ld;

    hipError_t e = alloc_device(h);
    if (e != hipSuccess) {
        free_device(h);
        delete h;
        return hip_fail(nullptr, e, "device allocation");
    }
    e = upload_meta(h);
    if (d->on_device) {
        // X gathered on the device into canonical order at the layout positions: only the
        // 4-byte source row of each device row crosses PCIe
        std::vector<int32_t> src((size_t)ld, -1);
        for (int64_t i = 0; i < n; ++i) src[(size_t)h->pos[i]] = (int32_t)h->perm[i];
        int32_t *d_src = nullptr;
        if (e == hipSuccess) e = hipMalloc(&d_src, sizeof(int32_t) * (size_t)ld);
        if (e == hipSuccess) e = hipMemcpy(d_src, src.data(), sizeof(int32_t) * (size_t)ld, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = (hipError_t)launch_gather_rows(d->x, d->ldx, d_src, nullptr, nullptr, nullptr, h->d_x, ld, (int)p,
                                               h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (d_src) (void)hipFree(d_src);
    } else {
        // X in canonical order at the layout positions, column by column
        std::vector<double> col(ld, 0.0);
        for (int64_t j = 0; j < p && e == hipSuccess; ++j) {
            const double *xj = d->x + j * d->ldx;
            for (int64_t i = 0; i < n; ++i) col[h->pos[i]] = xj[h->perm[i]];
            e = hipMemcpy(h->d_x + j * ld, col.data(), sizeof(double) * ld, hipMemcpyHostToDevice);
        }
    }
    // q_j = delta'X_j, summed on the device in a fixed order (the same for either source of X)
    if (e == hipSuccess) e = (hipError_t)launch_event_sums(h->d_x, ld, h->d_meta, h->q(), (int)p, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = upload_tables(h);
    if (e != hipSuccess) {
        free_device(h);
        delete h;
        return hip_fail(nullptr, e, "device upload");
    }
    *out = h;
    return COX_OK;
}

extern "C" int cox_init_indicator(cox_handle **out, int64_t n, int64_t p, const int64_t *col_ptr,
                                  const int32_t *row_idx, const double *time, const uint8_t *event,
                                  const int32_t *stratum, const cox_options *o)
{
    if (!out) return fail(nullptr, COX_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || p < 1) return fail(nullptr, COX_EINVAL, "need n >= 1 and p >= 1");
    if (n > (int64_t)kCountMask) return fail(nullptr, COX_EUNSUPPORTED, "n exceeds 2^29 - 1");
    if (p > kMaxCcdP) return fail(nullptr, COX_EUNSUPPORTED, "p > 12288 is not supported by the resident kernel");
    if (!col_ptr || !time || !event) return fail(nullptr, COX_EINVAL, "col_ptr, time and event are required");
    if (col_ptr[0] != 0) return fail(nullptr, COX_EINVAL, "col_ptr[0] must be 0");
    for (int64_t j = 0; j < p; ++j)
        if (col_ptr[j + 1] < col_ptr[j]) return fail(nullptr, COX_EINVAL, "col_ptr must be non-decreasing");
    const int64_t nnz = col_ptr[p];
    if (nnz > 0 && !row_idx) return fail(nullptr, COX_EINVAL, "row_idx is required");
    for (int64_t k = 0; k < nnz; ++k)
        if (row_idx[k] < 0 || row_idx[k] >= n) return fail(nullptr, COX_EINVAL, "row index out of range");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(time[i]) || event[i] > 1) return fail(nullptr, COX_EINVAL, "time must be finite, event 0 or 1");
    cox_options opt;
    if (o) opt = *o;
    else cox_default_options(&opt);
    {
        std::string msg;
        if (const int rc = check_options(opt, msg)) return fail(nullptr, rc, msg);
    }
    if (opt.mode != COX_CCD || opt.x_precision != COX_F64)
        return fail(nullptr, COX_EUNSUPPORTED, "indicator X runs COX_CCD fits in COX_F64");
    cox_handle *h = new cox_handle();
    h->n = n;
    h->p = p;
    h->opt = opt;
    h->opt.penalize = nullptr;
    h->stream = static_cast<hipStream_t>(opt.stream);
    (void)hipGetDevice(&h->device);
    canonical_order(n, time, event, stratum, h->perm, h->meta);
    h->gamma.assign((size_t)p, opt.gamma);
    if (o && o->penalize)
        for (int64_t j = 0; j < p; ++j) h->gamma[(size_t)j] = o->penalize[j] ? opt.gamma : 0.0;
    std::string err;
    const int rc = layout_for(h, err, false);
    if (rc != 0) {
        delete h;
        return fail(nullptr, rc, err);
    }
    const int ipt = h->shape.ipt;
    h->ldb = h->shape.ld / ipt;    // one unit per thread
    // bits at the layout positions: row r of the device layout is bit r % ipt of unit r / ipt
    std::vector<int64_t> dev_row((size_t)n);
    for (int64_t c = 0; c < n; ++c) dev_row[(size_t)h->perm[(size_t)c]] = h->pos[(size_t)c];
    const size_t unit = indicator_unit(ipt);
    std::vector<uint8_t> bits(unit * (size_t)h->ldb * (size_t)p, 0);
    std::vector<double> q((size_t)p, 0.0);
    for (int64_t j = 0; j < p; ++j) {
        double qj = 0.0;
        for (int64_t k = col_ptr[j]; k < col_ptr[j + 1]; ++k) {
            const int64_t i = row_idx[k];
            const int64_t r = dev_row[(size_t)i];
            const size_t u = (size_t)(j * h->ldb + r / ipt);
            const uint32_t bit = 1u << (r % ipt);
            if (unit == 1) {
                if (bits[u] & bit) continue;    // a repeated index sets the same entry once
                bits[u] = (uint8_t)(bits[u] | bit);
            } else {
                uint16_t w;
                std::memcpy(&w, &bits[2 * u], 2);
                if (w & bit) continue;
                w = (uint16_t)(w | bit);
                std::memcpy(&bits[2 * u], &w, 2);
            }
            if (event[i]) qj += 1.0;
        }
        q[(size_t)j] = qj;
    }
    hipError_t e = alloc_device(h);
    if (e != hipSuccess) {
        free_device(h);
        delete h;
        return hip_fail(nullptr, e, "device allocation");
    }
    e = upload_meta(h);
    if (e == hipSuccess) e = hipMemcpy(h->d_xbits, bits.data(), bits.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->q(), q.data(), sizeof(double) * p, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = upload_tables(h);
    if (e != hipSuccess) {
        free_device(h);
        delete h;
        return hip_fail(nullptr, e, "device upload");
    }
    *out = h;
    return COX_OK;
}

// delta'X_j of one sparse column (device rows ascending, values) in the order of the dense
// path's event sums (launch_event_sums: thread t of kEventSumThreads adds the event rows
// r = t (mod kEventSumThreads) in increasing r, then the partials meet in a halving tree), so
// that a sparse column's sum is bit-identical to the dense column's (its zeros add nothing).
static double event_sum_device_order(const std::vector<std::pair<int64_t, double>> &col,
                                     const std::vector<uint8_t> &ev_dev)
{
    std::vector<double> acc((size_t)kEventSumThreads, 0.0);
    for (const auto &e : col)
        if (ev_dev[(size_t)e.first]) acc[(size_t)(e.first % kEventSumThreads)] += e.second;
    for (int w = kEventSumThreads / 2; w > 0; w >>= 1)
        for (int t = 0; t < w; ++t) acc[(size_t)t] += acc[(size_t)(t + w)];
    return acc[0];
}

extern "C" int cox_init_sparse(cox_handle **out, int64_t n, int64_t p, const int64_t *col_ptr,
                               const int32_t *row_idx, const double *values, const double *time,
                               const uint8_t *event, const int32_t *stratum, const cox_options *o)
{
    if (!out) return fail(nullptr, COX_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || p < 1) return fail(nullptr, COX_EINVAL, "need n >= 1 and p >= 1");
    if (n > (int64_t)kCountMask) return fail(nullptr, COX_EUNSUPPORTED, "n exceeds 2^29 - 1");
    if (p > kMaxCcdP) return fail(nullptr, COX_EUNSUPPORTED, "p > 12288 is not supported by the resident kernel");
    if (!col_ptr || !time || !event) return fail(nullptr, COX_EINVAL, "col_ptr, time and event are required");
    if (col_ptr[0] != 0) return fail(nullptr, COX_EINVAL, "col_ptr[0] must be 0");
    for (int64_t j = 0; j < p; ++j)
        if (col_ptr[j + 1] < col_ptr[j]) return fail(nullptr, COX_EINVAL, "col_ptr must be non-decreasing");
    const int64_t nnz = col_ptr[p];
    if (nnz > 0 && (!row_idx || !values)) return fail(nullptr, COX_EINVAL, "row_idx and values are required");
    for (int64_t k = 0; k < nnz; ++k) {
        if (row_idx[k] < 0 || row_idx[k] >= n) return fail(nullptr, COX_EINVAL, "row index out of range");
        if (!std::isfinite(values[k])) return fail(nullptr, COX_EINVAL, "values must be finite");
    }
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(time[i]) || event[i] > 1) return fail(nullptr, COX_EINVAL, "time must be finite, event 0 or 1");
    cox_options opt;
    if (o) opt = *o;
    else cox_default_options(&opt);
    {
        std::string msg;
        if (const int rc = check_options(opt, msg)) return fail(nullptr, rc, msg);
    }
    if (opt.mode != COX_CCD || opt.x_precision != COX_F64)
        return fail(nullptr, COX_EUNSUPPORTED, "sparse X runs COX_CCD fits in COX_F64");
    cox_handle *h = new cox_handle();
    h->n = n;
    h->p = p;
    h->opt = opt;
    h->opt.penalize = nullptr;
    h->stream = static_cast<hipStream_t>(opt.stream);
    (void)hipGetDevice(&h->device);
    canonical_order(n, time, event, stratum, h->perm, h->meta);
    h->gamma.assign((size_t)p, opt.gamma);
    if (o && o->penalize)
        for (int64_t j = 0; j < p; ++j) h->gamma[(size_t)j] = o->penalize[j] ? opt.gamma : 0.0;
    std::string err;
    const int rc = layout_for(h, err, false);
    if (rc != 0) {
        delete h;
        return fail(nullptr, rc, err);
    }
    const int ipt = h->shape.ipt;
    h->ldb = h->shape.ld / ipt;    // one unit per thread
    const int64_t rows_per_wave = (int64_t)kWaveRows * ipt, nwaves = h->shape.ld / rows_per_wave;
    std::vector<int64_t> dev_row((size_t)n);
    for (int64_t c = 0; c < n; ++c) dev_row[(size_t)h->perm[(size_t)c]] = h->pos[(size_t)c];
    const size_t unit = indicator_unit(ipt);
    std::vector<uint8_t> bits(unit * (size_t)h->ldb * (size_t)p, 0);
    std::vector<double> q((size_t)p, 0.0), vals;
    std::vector<int64_t> voff((size_t)p, 0);
    std::vector<int32_t> woff((size_t)(p * nwaves), 0);
    std::vector<std::pair<int64_t, double>> col;
    std::vector<uint8_t> ev_dev((size_t)h->shape.ld, 0);
    for (int64_t c = 0; c < n; ++c) ev_dev[(size_t)h->pos[(size_t)c]] = event[h->perm[(size_t)c]];
    vals.reserve((size_t)nnz);
    for (int64_t j = 0; j < p; ++j) {
        // the column's nonzeros in device-row order (explicit zeros dropped)
        col.clear();
        for (int64_t k = col_ptr[j]; k < col_ptr[j + 1]; ++k)
            if (values[k] != 0.0) col.emplace_back(dev_row[(size_t)row_idx[k]], values[k]);
        std::sort(col.begin(), col.end(),
                  [](const std::pair<int64_t, double> &a, const std::pair<int64_t, double> &b) { return a.first < b.first; });
        for (size_t k = 1; k < col.size(); ++k)
            if (col[k].first == col[k - 1].first) {
                delete h;
                return fail(nullptr, COX_EINVAL, "a row index repeats within a column");
            }
        voff[(size_t)j] = (int64_t)vals.size();
        size_t k = 0;
        for (int64_t w = 0; w < nwaves; ++w) {
            woff[(size_t)(j * nwaves + w)] = (int32_t)k;
            while (k < col.size() && col[k].first < (w + 1) * rows_per_wave) ++k;
        }
        for (const auto &e : col) {
            const int64_t r = e.first;
            const size_t u = (size_t)(j * h->ldb + r / ipt);
            const uint32_t bit = 1u << (r % ipt);
            if (unit == 1) {
                bits[u] = (uint8_t)(bits[u] | bit);
            } else {
                uint16_t wd;
                std::memcpy(&wd, &bits[2 * u], 2);
                wd = (uint16_t)(wd | bit);
                std::memcpy(&bits[2 * u], &wd, 2);
            }
            vals.push_back(e.second);
        }
        q[(size_t)j] = event_sum_device_order(col, ev_dev);
    }
    hipError_t e = alloc_device(h);
    if (e == hipSuccess) e = hipMalloc(&h->d_xvals, sizeof(double) * std::max<size_t>(vals.size(), 1));
    if (e == hipSuccess) e = hipMalloc(&h->d_xvoff, sizeof(int64_t) * (size_t)p);
    if (e == hipSuccess) e = hipMalloc(&h->d_woff, sizeof(int32_t) * std::max<size_t>(woff.size(), 1));
    if (e != hipSuccess) {
        free_device(h);
        delete h;
        return hip_fail(nullptr, e, "device allocation");
    }
    e = upload_meta(h);
    if (e == hipSuccess) e = hipMemcpy(h->d_xbits, bits.data(), bits.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !vals.empty())
        e = hipMemcpy(h->d_xvals, vals.data(), sizeof(double) * vals.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->d_xvoff, voff.data(), sizeof(int64_t) * (size_t)p, hipMemcpyHostToDevice);
    if (e == hipSuccess && !woff.empty())
        e = hipMemcpy(h->d_woff, woff.data(), sizeof(int32_t) * woff.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->q(), q.data(), sizeof(double) * p, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = upload_tables(h);
    if (e != hipSuccess) {
        free_device(h);
        delete h;
        return hip_fail(nullptr, e, "device upload");
    }
    *out = h;
    return COX_OK;
}

// Canonical rows of the data set in which original row i appears count[i] times
// (copies numbered consecutively, original rows in order), derived from the
// parent's canonical order without sorting: copies of one row are adjacent and
// keep the parent's order.  The parent marks the last row of every tie group
// with events; the rows between two such marks are tie groups without events
// followed by that group, so the group's events are all the range's events and
// the child's mark goes on the last copy in the range.
static void resampled_order(const cox_handle *parent, const uint32_t *count, std::vector<int64_t> &perm,
                            std::vector<uint32_t> &meta, std::vector<int64_t> &from)
{
    const int64_t n = parent->n;
    std::vector<int64_t> first((size_t)n + 1, 0);   // first copy of original row i
    for (int64_t i = 0; i < n; ++i) first[(size_t)i + 1] = first[(size_t)i] + count[i];
    perm.clear();
    meta.clear();
    from.clear();
    bool head_pending = false;
    int64_t range_first = 0;    // first child row of the current range
    uint64_t range_events = 0;
    for (int64_t c = 0; c < n; ++c) {
        const uint32_t w = parent->meta[(size_t)c];
        if (w & kHeadBit) {
            head_pending = true;
            range_first = (int64_t)perm.size();
            range_events = 0;
        }
        const int64_t i = parent->perm[(size_t)c];
        const bool ev = (w & kEventBit) != 0u;
        for (uint32_t k = 0; k < count[i]; ++k) {
            perm.push_back(first[(size_t)i] + k);
            meta.push_back((head_pending ? kHeadBit : 0u) | (ev ? kEventBit : 0u));
            from.push_back(c);
            head_pending = false;
        }
        if (ev) range_events += count[i];
        if (w & kCountMask) {
            if ((int64_t)perm.size() > range_first && range_events > 0)
                meta.back() |= (uint32_t)range_events;
            range_first = (int64_t)perm.size();
            range_events = 0;
        }
    }
}

extern "C" int cox_init_resample(cox_handle **out, const cox_handle *parent, const uint32_t *count,
                                 const cox_options *o)
{
    if (!out) return fail(nullptr, COX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!parent || !count) return fail(nullptr, COX_EINVAL, "parent and count are required");
    if (parent->d_xvals)
        return fail(nullptr, COX_EUNSUPPORTED, "a handle on sparse X (cox_init_sparse) supports cox_fit and cox_evaluate only");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != parent->device) return fail(nullptr, COX_EINVAL, "the parent handle lives on another device");
    uint64_t total = 0;
    for (int64_t i = 0; i < parent->n; ++i) total += count[i];
    if (total < 1) return fail(nullptr, COX_EINVAL, "the resampled data set has no rows");
    if (total > (uint64_t)kCountMask) return fail(nullptr, COX_EUNSUPPORTED, "the resampled data set exceeds 2^29 - 1 rows");
    cox_options opt;
    if (o) opt = *o;
    else opt = parent->opt;
    {
        std::string msg;
        if (const int rc = check_options(opt, msg)) return fail(nullptr, rc, msg);
    }
    if (!parent->d_x && (opt.mode != COX_CCD || opt.x_precision != COX_F64))
        return fail(nullptr, COX_EUNSUPPORTED, "indicator X runs COX_CCD fits in COX_F64");
    cox_handle *h = new cox_handle();
    h->n = (int64_t)total;
    h->p = parent->p;
    h->opt = opt;
    h->opt.penalize = nullptr;
    h->stream = static_cast<hipStream_t>(opt.stream);
    h->device = parent->device;
    std::vector<int64_t> from;
    resampled_order(parent, count, h->perm, h->meta, from);
    if (o) {
        h->gamma.assign((size_t)h->p, opt.gamma);
        if (o->penalize)
            for (int64_t j = 0; j < h->p; ++j) h->gamma[(size_t)j] = o->penalize[j] ? opt.gamma : 0.0;
    } else {
        h->gamma = parent->gamma;
    }
    std::string err;
    const int rc = layout_for(h, err, parent->d_x != nullptr);
    if (rc != 0) {
        delete h;
        return fail(nullptr, rc, err);
    }
    const int64_t ld = h->shape.ld;
    if (parent->shape.ld > (int64_t)INT32_MAX) {
        delete h;
        return fail(nullptr, COX_EUNSUPPORTED, "parent layout too long for 32-bit row indices");
    }
    if (!parent->d_x) {
        if (h->shape.ipt == 0) {
            delete h;
            return fail(nullptr, COX_EUNSUPPORTED, "indicator X needs the persistent kernel's layout");
        }
        h->ldb = ld / h->shape.ipt;
    }
    // device row of the child -> device row of the parent (-1: padding)
    std::vector<int32_t> src((size_t)ld, -1);
    for (int64_t k = 0; k < h->n; ++k) src[(size_t)h->pos[(size_t)k]] = (int32_t)parent->pos[(size_t)from[(size_t)k]];
    hipError_t e = alloc_device(h);
    int32_t *d_src = nullptr;
    if (e == hipSuccess) e = hipMalloc(&d_src, sizeof(int32_t) * (size_t)ld);
    if (e != hipSuccess) {
        if (d_src) (void)hipFree(d_src);
        free_device(h);
        delete h;
        return hip_fail(nullptr, e, "device allocation");
    }
    e = upload_meta(h);
    if (e == hipSuccess) e = hipMemcpy(d_src, src.data(), sizeof(int32_t) * (size_t)ld, hipMemcpyHostToDevice);
    if (e == hipSuccess && parent->d_x) {
        e = (hipError_t)launch_gather_rows(parent->d_x, parent->shape.ld, d_src, nullptr, nullptr, nullptr, h->d_x, ld,
                                           (int)h->p, h->stream);
        if (e == hipSuccess) e = (hipError_t)launch_event_sums(h->d_x, ld, h->d_meta, h->q(), (int)h->p, h->stream);
    } else if (e == hipSuccess) {
        e = (hipError_t)launch_gather_bits(parent->d_xbits, parent->ldb, parent->shape.ipt, d_src, nullptr, nullptr,
                                           nullptr, h->d_xbits, h->ldb, h->shape.ipt, (int)h->p, h->stream);
        if (e == hipSuccess)
            e = (hipError_t)launch_event_sums_bits(h->d_xbits, h->ldb, h->shape.ipt, h->d_meta, h->q(), (int)h->p,
                                                   h->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(d_src);
    if (e == hipSuccess) e = upload_tables(h);
    if (e != hipSuccess) {
        free_device(h);
        delete h;
        return hip_fail(nullptr, e, "building the resampled data set");
    }
    *out = h;
    return COX_OK;
}

// Checks that (time, event, stratum) are the keys the parent's canonical order was built
// from: in the parent's order, the events match, each parent stratum carries one label
// (labels increasing from stratum to stratum), times do not increase within a stratum, and
// the tie groups with events -- runs of equal times -- end where the parent's row words say,
// with the same event counts.  O(n); returns nullptr or a message.
static const char *same_keys_as_parent(const cox_handle *parent, const double *time, const uint8_t *event,
                                       const int32_t *stratum)
{
    const int64_t n = parent->n;
    uint32_t group_events = 0;
    for (int64_t c = 0; c < n; ++c) {
        const uint32_t w = parent->meta[(size_t)c];
        const int64_t r = parent->perm[(size_t)c];
        if (((w & kEventBit) != 0u) != (event[r] != 0)) return "event is not the data the parent was built from";
        if (c > 0) {
            const int64_t rp = parent->perm[(size_t)(c - 1)];
            const int32_t sp = stratum ? stratum[rp] : 0, sc = stratum ? stratum[r] : 0;
            if ((w & kHeadBit) ? !(sc > sp) : (sc != sp)) return "stratum is not the data the parent was built from";
            if (!(w & kHeadBit) && time[r] > time[rp]) return "time is not the data the parent was built from";
        } else if (!(w & kHeadBit)) {
            return "the parent's layout has no head row";
        }
        group_events += event[r] ? 1u : 0u;
        const bool last = c + 1 == n || (parent->meta[(size_t)(c + 1)] & kHeadBit) != 0u ||
                          time[parent->perm[(size_t)(c + 1)]] != time[r];
        if ((w & kCountMask) != (last ? group_events : 0u)) return "time is not the data the parent was built from";
        if (last) group_events = 0;
    }
    return nullptr;
}

extern "C" int cox_init_intervals(cox_handle **out, const cox_handle *parent, const double *time,
                                  const uint8_t *event, const int32_t *stratum, int ncuts, const double *cuts,
                                  const uint8_t *tv_coef, const cox_options *o)
{
    if (!out) return fail(nullptr, COX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!parent) return fail(nullptr, COX_EINVAL, "parent is NULL");
    if (parent->d_xvals)
        return fail(nullptr, COX_EUNSUPPORTED, "a handle on sparse X (cox_init_sparse) supports cox_fit and cox_evaluate only");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != parent->device) return fail(nullptr, COX_EINVAL, "the parent handle lives on another device");
    const int64_t n = parent->n, p = parent->p;
    if (!time || !event) return fail(nullptr, COX_EINVAL, "time and event are required");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(time[i]) || event[i] > 1) return fail(nullptr, COX_EINVAL, "time must be finite, event 0 or 1");
    if (const char *bad = same_keys_as_parent(parent, time, event, stratum))
        return fail(nullptr, COX_EINVAL, bad);
    cox_options opt;
    if (o) opt = *o;
    else opt = parent->opt;
    {
        std::string msg;
        if (const int rc = check_options(opt, msg)) return fail(nullptr, rc, msg);
    }
    if (!parent->d_x && (opt.mode != COX_CCD || opt.x_precision != COX_F64))
        return fail(nullptr, COX_EUNSUPPORTED, "indicator X runs COX_CCD fits in COX_F64");
    IntervalRows rows;
    try {
        const int rc = interval_rows(n, time, event, stratum, ncuts, cuts, tv_coef, p, rows);
        if (rc != COX_OK) return fail(nullptr, rc, "bad cuts, or too many augmented rows or strata");
    } catch (const std::bad_alloc &) {
        return fail(nullptr, COX_ENOMEM, "host memory for the augmented rows");
    }
    const int64_t naug = (int64_t)rows.time.size(), paug = (int64_t)rows.col_source.size();
    if (naug > (int64_t)kCountMask) return fail(nullptr, COX_EUNSUPPORTED, "more than 2^29 - 1 augmented rows");
    if (paug > kMaxCcdP || (opt.mode == COX_NEWTON_REFINE && paug > kMaxNewtonP))
        return fail(nullptr, COX_EUNSUPPORTED, "too many augmented columns (12288 for COX_CCD, 4096 for Newton)");
    cox_handle *h = new cox_handle();
    h->n = naug;
    h->p = paug;
    h->opt = opt;
    h->opt.penalize = nullptr;
    h->stream = static_cast<hipStream_t>(opt.stream);
    h->device = parent->device;
    canonical_order(naug, rows.time.data(), rows.event.data(), rows.stratum.data(), h->perm, h->meta);
    h->gamma.assign((size_t)paug, opt.gamma);
    if (o) {
        if (o->penalize)
            for (int64_t c = 0; c < paug; ++c) h->gamma[(size_t)c] = o->penalize[c] ? opt.gamma : 0.0;
    } else {
        for (int64_t c = 0; c < paug; ++c) h->gamma[(size_t)c] = parent->gamma[(size_t)rows.col_source[(size_t)c]];
    }
    std::string err;
    const int rc = layout_for(h, err, parent->d_x != nullptr);
    if (rc != 0) {
        delete h;
        return fail(nullptr, rc, err);
    }
    const int64_t ld = h->shape.ld;
    if (parent->shape.ld > (int64_t)INT32_MAX) {
        delete h;
        return fail(nullptr, COX_EUNSUPPORTED, "parent layout too long for 32-bit row indices");
    }
    if (!parent->d_x) {
        if (h->shape.ipt == 0) {
            delete h;
            return fail(nullptr, COX_EUNSUPPORTED, "indicator X needs the persistent kernel's layout");
        }
        h->ldb = ld / h->shape.ipt;
    }
    // maps: [0, ld) source row, [ld, 2 ld) interval of each device row, then column source and interval
    std::vector<int32_t> maps((size_t)(2 * ld + 2 * paug), -1);
    {
        std::vector<int64_t> canon_of((size_t)n);
        for (int64_t c = 0; c < n; ++c) canon_of[(size_t)parent->perm[(size_t)c]] = c;
        for (int64_t k = 0; k < naug; ++k) {
            const int64_t a = h->perm[(size_t)k];
            const int64_t r = h->pos[(size_t)k];
            maps[(size_t)r] = (int32_t)parent->pos[(size_t)canon_of[(size_t)rows.row_subject[(size_t)a]]];
            maps[(size_t)(ld + r)] = rows.row_interval[(size_t)a];
        }
        std::copy(rows.col_source.begin(), rows.col_source.end(), maps.begin() + 2 * ld);
        std::copy(rows.col_interval.begin(), rows.col_interval.end(), maps.begin() + 2 * ld + paug);
    }
    hipError_t e = alloc_device(h);
    int32_t *d_maps = nullptr;
    if (e == hipSuccess) e = hipMalloc(&d_maps, sizeof(int32_t) * maps.size());
    if (e != hipSuccess) {
        if (d_maps) (void)hipFree(d_maps);
        free_device(h);
        delete h;
        return hip_fail(nullptr, e, "device allocation");
    }
    e = upload_meta(h);
    if (e == hipSuccess) e = hipMemcpy(d_maps, maps.data(), sizeof(int32_t) * maps.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && parent->d_x) {
        e = (hipError_t)launch_gather_rows(parent->d_x, parent->shape.ld, d_maps, d_maps + ld, d_maps + 2 * ld,
                                           d_maps + 2 * ld + paug, h->d_x, ld, (int)paug, h->stream);
        if (e == hipSuccess) e = (hipError_t)launch_event_sums(h->d_x, ld, h->d_meta, h->q(), (int)paug, h->stream);
    } else if (e == hipSuccess) {
        e = (hipError_t)launch_gather_bits(parent->d_xbits, parent->ldb, parent->shape.ipt, d_maps, d_maps + ld,
                                           d_maps + 2 * ld, d_maps + 2 * ld + paug, h->d_xbits, h->ldb, h->shape.ipt,
                                           (int)paug, h->stream);
        if (e == hipSuccess)
            e = (hipError_t)launch_event_sums_bits(h->d_xbits, h->ldb, h->shape.ipt, h->d_meta, h->q(), (int)paug,
                                                   h->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(d_maps);
    if (e == hipSuccess) e = upload_tables(h);
    if (e != hipSuccess) {
        free_device(h);
        delete h;
        return hip_fail(nullptr, e, "building the interval-stratified data set");
    }
    h->subject = std::move(rows.row_subject);
    *out = h;
    return COX_OK;
}

extern "C" int cox_set_penalty(cox_handle *h, double gamma, const uint8_t *penalize)
{
    if (!h) return fail(nullptr, COX_EINVAL, "handle is NULL");
    if (!(gamma >= 0.0) || !std::isfinite(gamma)) return fail(h, COX_EINVAL, "gamma must be finite and >= 0");
    std::vector<double> g((size_t)h->p, gamma);
    if (penalize)
        for (int64_t j = 0; j < h->p; ++j) g[(size_t)j] = penalize[j] ? gamma : 0.0;
    const hipError_t e = hipMemcpy(h->gam(), g.data(), sizeof(double) * h->p, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(h, e, "uploading the l1 weights");
    h->gamma.swap(g);
    h->opt.gamma = gamma;
    return COX_OK;
}

// Run the persistent kernel in `mode` over columns [j0, j1) starting from beta (host, p).
static int run_kernel(cox_handle *h, int mode, int j0, int j1, const double *beta_host, double *result)
{
    (void)hipSetDevice(h->device);
    if (h->shape.ipt == 0)
        return fail(h, COX_EUNSUPPORTED,
                    "n exceeds the register-resident capacity of the persistent kernel: this handle supports "
                    "cox_fit (by Newton steps), cox_evaluate and cox_evaluate_full only");
    hipError_t e;
    if (beta_host) e = hipMemcpyAsync(h->beta(), beta_host, sizeof(double) * h->p, hipMemcpyHostToDevice, h->stream);
    else e = hipMemsetAsync(h->beta(), 0, sizeof(double) * h->p, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->result(), 0, sizeof(double) * kResultSlots, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "staging beta");
    CcdLaunch L;
    L.x = h->d_x;
    L.xbits = h->d_xbits;
    L.ldb = h->ldb;
    L.xvals = h->d_xvals;
    L.xvoff = h->d_xvoff;
    L.woff = h->d_woff;
    L.nwaves = h->shape.ipt ? h->shape.ld / ((int64_t)kWaveRows * h->shape.ipt) : 0;
    L.meta = h->d_meta;
    L.q = h->q();
    L.gamma = h->gam();
    L.trust = h->d_trust;
    L.exp_tab = h->exp_tab();
    L.n = h->n;
    L.p = (int)h->p;
    L.mode = mode;
    L.efron = h->opt.ties == COX_EFRON ? 1 : 0;
    L.wave = h->shape.wave ? 1 : 0;
    L.j0 = j0;
    L.j1 = j1;
    L.max_sweeps = h->opt.max_iter;
    L.tol = h->opt.tol;
    L.beta = h->beta();
    L.g1 = h->g1();
    L.g2 = h->g2();
    L.m2 = h->m2();
    L.result = h->result();
    carve_sync_scratch(h->d_sync, h->shape.grid, L);
    int rc = launch_ccd(h->shape, L, h->stream, h->ev0, h->ev1);
    if (rc != (int)hipSuccess) return hip_fail(h, (hipError_t)rc, "kernel launch");
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_fail(h, e, "kernel execution");
    (void)hipEventElapsedTime(&h->last_kernel_ms, h->ev0, h->ev1);
    h->prof = cox_profile{};
    h->prof.kernel_ms = h->last_kernel_ms;
    uint32_t ctl[2] = {0, 0};
    if ((e = hipMemcpy(ctl, L.ctl, sizeof(ctl), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(h, e, "reading control words");
    if ((e = hipMemcpy(result, h->result(), sizeof(double) * kResultSlots, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(h, e, "reading results");
    if (ctl[0] != 0u || result[kResCompleted] != 1.0)
        return fail(h, COX_EDEVICE, "device-side synchronisation timed out; results are not valid");
    if (result[kResNumeric] != 0.0)
        return fail(h, COX_ENUMERIC, "a risk-set sum left the FP64 normal range after the global shift");
    return COX_OK;
}

extern "C" int cox_fit(cox_handle *h, const double *beta0, double *beta_out, cox_fit_info *info)
{
    if (!h) return fail(nullptr, COX_EINVAL, "handle is NULL");
    if (!beta_out) return fail(h, COX_EINVAL, "beta_out is NULL");
    if (beta0)
        for (int64_t j = 0; j < h->p; ++j)
            if (!std::isfinite(beta0[j])) return fail(h, COX_EINVAL, "beta0 is not finite");
    if (info) info->fallback = 0;
    if (h->opt.mode == COX_NEWTON_REFINE) return newton_fit(h, beta0, beta_out, info);
    if (h->shape.ipt == 0) {
        // more rows than the persistent kernel holds (dense X): (proximal) Newton steps on the
        // full evaluation reach the same optimum
        const int rc2 = newton_fit(h, beta0, beta_out, info);
        if (info && (rc2 == COX_OK || rc2 == COX_NOT_CONVERGED)) info->fallback = 2;
        return rc2;
    }
    double res[kResultSlots];
    int rc = run_kernel(h, kModeFit, 0, (int)h->p, beta0, res);
    if (rc == COX_ENUMERIC && h->d_x) {
        // the one shift of the persistent kernel cannot hold exp(X beta) in range: finish on the
        // full evaluation (running-maximum scans), Newton or proximal Newton steps in FP64
        const int rc2 = newton_fit(h, beta0, beta_out, info);
        if (rc2 == COX_OK || rc2 == COX_NOT_CONVERGED) {
            if (info) info->fallback = 1;
            return rc2;
        }
        return rc2;
    }
    if (rc != COX_OK && rc != COX_ENUMERIC) return rc;
    hipError_t e = hipMemcpy(beta_out, h->beta(), sizeof(double) * h->p, hipMemcpyDeviceToHost);
    std::vector<double> g(h->p);
    if (e == hipSuccess) e = hipMemcpy(g.data(), h->g1(), sizeof(double) * h->p, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "reading beta");
    const bool converged = res[kResConverged] == 1.0;
    if (rc == COX_OK && !converged) rc = COX_NOT_CONVERGED;
    if (info) {
        info->status = rc;
        info->iters = (int)res[kResSweeps];
        info->coord_evals = (int64_t)res[kResSweeps] * h->p;
        info->objective = res[kResObjective];
        info->last_step = res[kResLastStep];
        info->n_pinned = (int)res[kResPinned];
        double kkt = 0.0;
        for (int64_t j = 0; j < h->p; ++j) {
            const double gj = g[j], gm = h->gamma[j], b = beta_out[j];
            double r;
            if (gm <= 0.0) r = std::fabs(gj);
            else if (b != 0.0) r = std::fabs(gj + (b > 0 ? gm : -gm));
            else r = std::max(std::fabs(gj) - gm, 0.0);
            kkt = std::max(kkt, r);
        }
        info->kkt_inf = kkt;
    }
    return rc;
}

// -log partial likelihood (Eq. strat_l, no penalty) of h's data at beta: the persistent
// kernel's evaluation of one coordinate, or the full evaluation on a Newton handle.
static int neg_loglik(cox_handle *h, const double *beta, double *nll)
{
    if (h->opt.mode == COX_NEWTON_REFINE || h->shape.ipt == 0) {
        double obj = 0.0;
        const int rc = cox_evaluate_full(h, beta, &obj, nullptr, nullptr, nullptr);
        if (rc != COX_OK) return rc;
        double pen = 0.0;
        for (int64_t j = 0; j < h->p; ++j) pen += h->gamma[(size_t)j] * std::fabs(beta[j]);
        *nll = obj - pen;
        return COX_OK;
    }
    double res[kResultSlots];
    const int rc = run_kernel(h, kModeEval, 0, 1, beta, res);
    if (rc != COX_OK) return rc;
    *nll = res[kResObjective];
    return COX_OK;
}

// The argument checks of a cross-validation; 0 or a COX_* code with the message set on h.
static int check_folds(cox_handle *h, int nfolds, const int32_t *fold, int ngamma, const double *gammas,
                       const double *cvl)
{
    if (nfolds < 2 || !fold) return fail(h, COX_EINVAL, "need nfolds >= 2 and a fold for every row");
    if (ngamma < 1 || !gammas || !cvl) return fail(h, COX_EINVAL, "need ngamma >= 1, gammas and cvl");
    for (int g = 0; g < ngamma; ++g)
        if (!(gammas[g] >= 0.0) || !std::isfinite(gammas[g])) return fail(h, COX_EINVAL, "gamma must be finite and >= 0");
    std::vector<int64_t> size((size_t)nfolds, 0);
    for (int64_t i = 0; i < h->n; ++i) {
        if (fold[i] < 0 || fold[i] >= nfolds) return fail(h, COX_EINVAL, "fold index out of range");
        ++size[(size_t)fold[i]];
    }
    for (int k = 0; k < nfolds; ++k)
        if (size[(size_t)k] == 0 || size[(size_t)k] == h->n) return fail(h, COX_EINVAL, "every fold must hold some rows, and not all");
    if (!h->subject.empty()) {
        // interval-stratified rows: a subject's rows are held out together
        int64_t ns = 0;
        for (int64_t s : h->subject) ns = std::max(ns, s + 1);
        std::vector<int32_t> of((size_t)ns, -1);
        for (int64_t i = 0; i < h->n; ++i) {
            int32_t &f = of[(size_t)h->subject[(size_t)i]];
            if (f < 0) f = fold[i];
            else if (f != fold[i]) return fail(h, COX_EINVAL, "rows of one subject fall in different folds");
        }
    }
    return COX_OK;
}

extern "C" int cox_cross_validate(cox_handle *h, int nfolds, const int32_t *fold, int ngamma, const double *gammas,
                                  const uint8_t *penalize, double *cvl, double *betas, int *status)
{
    if (!h) return fail(nullptr, COX_EINVAL, "handle is NULL");
    if (const int rc = check_folds(h, nfolds, fold, ngamma, gammas, cvl)) return rc;
    const int64_t p = h->p;
    std::fill(cvl, cvl + ngamma, 0.0);
    bool all_converged = true;
    std::vector<uint32_t> keep((size_t)h->n);
    std::vector<double> beta((size_t)p), prev((size_t)p);
    for (int k = 0; k < nfolds; ++k) {
        for (int64_t i = 0; i < h->n; ++i) keep[(size_t)i] = fold[i] != k ? 1u : 0u;
        cox_options o = h->opt;
        o.gamma = gammas[0];
        o.penalize = penalize;
        cox_handle *c = nullptr;
        int rc = cox_init_resample(&c, h, keep.data(), &o);
        if (rc != COX_OK) return fail(h, rc, std::string("fold training set: ") + cox_last_error(nullptr));
        std::fill(prev.begin(), prev.end(), 0.0);
        for (int g = 0; g < ngamma && rc >= 0; ++g) {
            rc = cox_set_penalty(c, gammas[g], penalize);
            cox_fit_info info{};
            if (rc == COX_OK) rc = cox_fit(c, prev.data(), beta.data(), &info);
            if (rc < 0) break;
            if (rc != COX_OK) all_converged = false;
            if (status) status[(size_t)k * ngamma + g] = rc;
            double nll_train = 0.0, nll_full = 0.0;
            int rc2 = neg_loglik(c, beta.data(), &nll_train);
            if (rc2 == COX_OK) rc2 = neg_loglik(h, beta.data(), &nll_full);
            if (rc2 != COX_OK) {
                rc = rc2;
                break;
            }
            cvl[g] += nll_train - nll_full;    // l(beta) - l_{-k}(beta), l = log partial likelihood
            if (betas) std::copy(beta.begin(), beta.end(), betas + ((size_t)k * ngamma + g) * p);
            prev = beta;
            rc = COX_OK;
        }
        const std::string cerr = rc < 0 ? c->err : std::string();
        cox_release(c);
        if (rc < 0) return fail(h, rc, "fold " + std::to_string(k) + ": " + cerr);
    }
    return all_converged ? COX_OK : COX_NOT_CONVERGED;
}

extern "C" int cox_cross_validate_served(cox_handle *h, cox_server *srv, const cox_data *d, int nfolds,
                                         const int32_t *fold, int ngamma, const double *gammas,
                                         const uint8_t *penalize, double *cvl, double *betas, int *status)
{
    if (!h) return fail(nullptr, COX_EINVAL, "handle is NULL");
    if (!srv || !d) return fail(h, COX_EINVAL, "server and data are required");
    if (d->on_device) return fail(h, COX_EINVAL, "the fold requests are built from host data");
    if (d->n != h->n || d->p != h->p || !h->subject.empty())
        return fail(h, COX_EINVAL, "d must be the data the handle was made from by cox_init");
    if (const char *bad = check_data(d->n, d->p, d->ldx, d->x, d->time, d->event)) return fail(h, COX_EINVAL, bad);
    if (const int rc = check_folds(h, nfolds, fold, ngamma, gammas, cvl)) return rc;
    const int64_t n = h->n, p = h->p;
    // each fold's training rows, copied once (column-major X, keys)
    struct Train {
        int64_t n = 0;
        std::vector<double> x, t;
        std::vector<uint8_t> e;
        std::vector<int32_t> st;
        cox_data data{};
    };
    std::vector<Train> tr((size_t)nfolds);
    for (int k = 0; k < nfolds; ++k) {
        Train &T = tr[(size_t)k];
        for (int64_t i = 0; i < n; ++i) T.n += fold[i] != k ? 1 : 0;
        T.x.resize((size_t)(T.n * p));
        T.t.resize((size_t)T.n);
        T.e.resize((size_t)T.n);
        if (d->stratum) T.st.resize((size_t)T.n);
        int64_t r = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (fold[i] == k) continue;
            for (int64_t j = 0; j < p; ++j) T.x[(size_t)(j * T.n + r)] = d->x[j * d->ldx + i];
            T.t[(size_t)r] = d->time[i];
            T.e[(size_t)r] = d->event[i];
            if (d->stratum) T.st[(size_t)r] = d->stratum[i];
            ++r;
        }
        T.data.n = T.n;
        T.data.p = p;
        T.data.x = T.x.data();
        T.data.ldx = T.n;
        T.data.time = T.t.data();
        T.data.event = T.e.data();
        T.data.stratum = d->stratum ? T.st.data() : nullptr;
    }
    // the fits: every fold at one weight in one batch, warm-started from the previous weight's fits
    std::vector<double> all((size_t)nfolds * ngamma * p, 0.0);
    std::vector<int> stat((size_t)nfolds * ngamma, COX_OK);
    std::vector<uint64_t> tickets((size_t)nfolds);
    for (int g = 0; g < ngamma; ++g) {
        for (int k = 0; k < nfolds; ++k) {
            cox_fit_request r{};
            r.gamma = gammas[g];
            r.penalize = penalize;
            r.beta0 = g > 0 ? all.data() + ((size_t)k * ngamma + g - 1) * p : nullptr;
            const int rc = cox_server_submit_fit(srv, &tr[(size_t)k].data, COX_SUBMIT_BORROW, &r, &tickets[(size_t)k]);
            if (rc != COX_OK) return fail(h, rc, std::string("fold request: ") + cox_server_last_error(srv));
        }
        for (int k = 0; k < nfolds; ++k) {
            int rc = cox_server_wait(srv, tickets[(size_t)k], -1.0);
            cox_fit_info info{};
            if (rc == COX_OK)
                rc = cox_server_poll(srv, tickets[(size_t)k], all.data() + ((size_t)k * ngamma + g) * p, &info, nullptr);
            if (rc != COX_OK) return fail(h, rc, std::string("fold fit: ") + cox_server_last_error(srv));
            if (info.status < 0) return fail(h, info.status, "fold " + std::to_string(k) + " fit failed");
            stat[(size_t)k * ngamma + g] = info.status;
        }
    }
    // the criterion: l(beta_{-k}) - l_{-k}(beta_{-k}) from the full handle and a training handle per fold
    std::fill(cvl, cvl + ngamma, 0.0);
    std::vector<uint32_t> keep((size_t)n);
    bool all_converged = true;
    for (int k = 0; k < nfolds; ++k) {
        for (int64_t i = 0; i < n; ++i) keep[(size_t)i] = fold[i] != k ? 1u : 0u;
        cox_options o = h->opt;
        o.mode = COX_CCD;
        o.x_precision = COX_F64;
        o.gamma = 0.0;
        o.penalize = nullptr;
        cox_handle *c = nullptr;
        int rc = cox_init_resample(&c, h, keep.data(), &o);
        if (rc != COX_OK) return fail(h, rc, std::string("fold training set: ") + cox_last_error(nullptr));
        for (int g = 0; g < ngamma && rc == COX_OK; ++g) {
            const double *beta = all.data() + ((size_t)k * ngamma + g) * p;
            double nll_train = 0.0, nll_full = 0.0;
            rc = neg_loglik(c, beta, &nll_train);
            if (rc == COX_OK) rc = neg_loglik(h, beta, &nll_full);
            if (rc == COX_OK) cvl[g] += nll_train - nll_full;
        }
        const std::string cerr = rc != COX_OK ? c->err : std::string();
        cox_release(c);
        if (rc != COX_OK) return fail(h, rc, "fold " + std::to_string(k) + ": " + cerr);
    }
    for (size_t q = 0; q < stat.size(); ++q) {
        if (stat[q] != COX_OK) all_converged = false;
        if (status) status[q] = stat[q];
    }
    if (betas) std::copy(all.begin(), all.end(), betas);
    return all_converged ? COX_OK : COX_NOT_CONVERGED;
}

extern "C" int cox_bootstrap(cox_handle *h, int nrep, const uint32_t *counts, const double *beta0, double *betas,
                             int *status)
{
    if (!h) return fail(nullptr, COX_EINVAL, "handle is NULL");
    if (nrep < 1 || !counts || !betas) return fail(h, COX_EINVAL, "need nrep >= 1, counts and betas");
    const int64_t n = h->n, p = h->p;
    bool all_converged = true;
    for (int b = 0; b < nrep; ++b) {
        cox_handle *c = nullptr;
        int rc = cox_init_resample(&c, h, counts + (size_t)b * n, nullptr);
        if (rc != COX_OK) return fail(h, rc, "replicate " + std::to_string(b) + ": " + cox_last_error(nullptr));
        cox_fit_info info{};
        rc = cox_fit(c, beta0, betas + (size_t)b * p, &info);
        const std::string cerr = rc < 0 ? c->err : std::string();
        cox_release(c);
        if (rc < 0) return fail(h, rc, "replicate " + std::to_string(b) + ": " + cerr);
        if (status) status[b] = rc;
        if (rc != COX_OK) all_converged = false;
    }
    return all_converged ? COX_OK : COX_NOT_CONVERGED;
}

extern "C" int cox_evaluate(cox_handle *h, const double *beta, double *objective, double *grad,
                            double *hess_diag)
{
    if (!h) return fail(nullptr, COX_EINVAL, "handle is NULL");
    if (!beta) return fail(h, COX_EINVAL, "beta is NULL");
    if (h->shape.ipt == 0 && h->d_x)   // beyond the persistent kernel: the full evaluation
        return cox_evaluate_full(h, beta, objective, grad, hess_diag, nullptr);
    double res[kResultSlots];
    int rc = run_kernel(h, kModeEval, 0, (int)h->p, beta, res);
    if (rc == COX_ENUMERIC && h->d_x) {
        // beyond the one shift's range: the full evaluation (running-maximum scans) gives the
        // same objective, gradient and diagonal Hessian
        return cox_evaluate_full(h, beta, objective, grad, hess_diag, nullptr);
    }
    if (rc != COX_OK) return rc;
    hipError_t e = hipSuccess;
    if (grad) e = hipMemcpy(grad, h->g1(), sizeof(double) * h->p, hipMemcpyDeviceToHost);
    if (hess_diag && e == hipSuccess) e = hipMemcpy(hess_diag, h->g2(), sizeof(double) * h->p, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "reading gradient");
    if (objective) {
        double pen = 0.0;
        for (int64_t j = 0; j < h->p; ++j) pen += h->gamma[j] * std::fabs(beta[j]);
        *objective = res[kResObjective] + pen;
    }
    return COX_OK;
}

extern "C" int cox_coordinate(cox_handle *h, const double *beta, int64_t j, double *out)
{
    if (!h) return fail(nullptr, COX_EINVAL, "handle is NULL");
    if (!beta || !out) return fail(h, COX_EINVAL, "beta and out are required");
    if (j < 0 || j >= h->p) return fail(h, COX_EINVAL, "column index out of range");
    double res[kResultSlots];
    int rc = run_kernel(h, kModeEval, (int)j, (int)j + 1, beta, res);
    if (rc != COX_OK) return rc;
    double v[3];
    hipError_t e = hipMemcpy(&v[0], h->g1() + j, sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&v[1], h->g2() + j, sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&v[2], h->m2() + j, sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "reading coordinate");
    out[0] = v[0];
    out[1] = v[1];
    out[2] = res[kResObjective];
    out[3] = v[2];
    return COX_OK;
}

extern "C" int cox_layout(const cox_handle *h, int64_t *perm, uint32_t *meta)
{
    if (!h) return COX_EINVAL;
    if (perm) std::memcpy(perm, h->perm.data(), sizeof(int64_t) * h->n);
    if (meta) std::memcpy(meta, h->meta.data(), sizeof(uint32_t) * h->n);
    return COX_OK;
}

extern "C" int cox_canonical_order(int64_t n, const double *time, const uint8_t *event, const int32_t *stratum,
                                   int64_t *perm, uint32_t *meta)
{
    if (n < 1 || !perm || !meta) return COX_EINVAL;
    if (n > (int64_t)kCountMask || !time || !event) return COX_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(time[i]) || event[i] > 1) return COX_EINVAL;
    std::vector<int64_t> pv;
    std::vector<uint32_t> mv;
    canonical_order(n, time, event, stratum, pv, mv);
    std::memcpy(perm, pv.data(), sizeof(int64_t) * n);
    std::memcpy(meta, mv.data(), sizeof(uint32_t) * n);
    return COX_OK;
}

extern "C" int cox_last_profile(const cox_handle *h, cox_profile *out)
{
    if (!h || !out) return COX_EINVAL;
    *out = h->prof;
    return COX_OK;
}

extern "C" int cox_shape(const cox_handle *h, int64_t *n, int64_t *p, int64_t *ld)
{
    if (!h) return COX_EINVAL;
    if (n) *n = h->n;
    if (p) *p = h->p;
    if (ld) *ld = h->shape.ld;
    return COX_OK;
}

extern "C" int cox_last_kernel_ms(const cox_handle *h, double *ms)
{
    if (!h || !ms) return COX_EINVAL;
    *ms = h->last_kernel_ms;
    return COX_OK;
}

extern "C" int cox_segscan_f64(const double *a, const uint8_t *head, double *b, int64_t n, void *stream)
{
    if (n > 0x7fffffffLL) return COX_EUNSUPPORTED;
    return segscan_f64(a, head, b, n, static_cast<hipStream_t>(stream));
}

extern "C" int cox_segscan_f64_noalloc(const double *a, const uint8_t *head, double *b, int64_t n, void *stream)
{
    if (n > 0x7fffffffLL) return COX_EUNSUPPORTED;
    return segscan_f64_noalloc(a, head, b, n, static_cast<hipStream_t>(stream));
}

extern "C" void cox_release(cox_handle *h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    free_device(h);
    delete h;
}

extern "C" const char *cox_last_error(const cox_handle *h)
{
    return h ? h->err.c_str() : g_init_error.c_str();
}
