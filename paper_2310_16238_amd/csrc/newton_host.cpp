// newton_host.cpp -- full evaluation and the Newton / iterative-refinement fit
// (host side; kernels in newton.hip and contraction.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "handle.h"
#include "internal.h"
#include "newton.h"

using namespace coxmi;

namespace {

constexpr int kScalSlots = 8;

double *nrow(const NewtonState &s, int64_t ld, int k) { return s.rows + (int64_t)k * ld; }

double elapsed_ms(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.0f;
    return hipEventElapsedTime(&ms, a, b) == hipSuccess ? (double)ms : 0.0;
}

template <typename T>
hipError_t dalloc(T **p, size_t bytes)
{
    return hipMalloc(reinterpret_cast<void **>(p), bytes);
}

// xbar (Z) is kept in BF16 for both reduced-precision modes
bool lowp(int prec) { return prec == COX_BF16 || prec == COX_FP8_E4M3; }
size_t ztype_bytes(int prec) { return lowp(prec) ? 2 : 8; }

int newton_setup(cox_handle *h)
{
    if (h->p > kMaxNewtonP)
        return handle_fail(h, COX_EUNSUPPORTED, "the full evaluation and Newton fits support p <= 4096");
    if (h->opt.x_precision == COX_FP8_E4M3 && h->p > kMaxFp8P)
        return handle_fail(h, COX_EUNSUPPORTED, "the FP8 contraction supports p <= 4096");
    if (!h->d_x)
        return handle_fail(h, COX_EUNSUPPORTED,
                           "a handle on indicator X runs the CCD path only (cox_fit in COX_CCD mode, cox_evaluate, "
                           "cox_coordinate)");
    NewtonState &s = h->nt;
    if (s.ready) return COX_OK;
    const int64_t ld = h->shape.ld, n = h->n;
    const int p = (int)h->p;
    std::vector<int32_t> gidx(ld, -1);
    std::vector<uint8_t> head(ld, 1);   // padding rows are one-row strata
    int64_t G = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (h->meta[i] & kCountMask) gidx[h->pos[i]] = (int32_t)G++;
        head[h->pos[i]] = (h->meta[i] & kHeadBit) ? 1 : 0;
    }
    s.n_groups = G;
    // Efron: the event rows of every group with two or more events, and for every event row
    // the end row of its group (a group's events are the event rows after the previous
    // event-group end of the stratum, up to its own end)
    s.efron = h->opt.ties == COX_EFRON;
    std::vector<int32_t> gidx2, gend, me_ptr, me_row, me_end;
    if (s.efron) {
        gidx2.assign(ld, -1);
        gend.assign(ld, -1);
        me_ptr.push_back(0);
        std::vector<int32_t> pending;
        for (int64_t i = 0; i < n; ++i) {
            if (h->meta[i] & kHeadBit) pending.clear();
            if (h->meta[i] & kEventBit) pending.push_back((int32_t)h->pos[i]);
            const uint32_t d = h->meta[i] & kCountMask;
            if (d == 0u) continue;
            if (pending.size() != d) return handle_fail(h, COX_EDEVICE, "inconsistent tie groups");
            const int32_t e = (int32_t)h->pos[i];
            for (int32_t r : pending) gend[(size_t)r] = e;
            if (d >= 2u) {
                gidx2[(size_t)e] = (int32_t)me_end.size();
                me_end.push_back(e);
                me_row.insert(me_row.end(), pending.begin(), pending.end());
                me_ptr.push_back((int32_t)me_row.size());
            }
            pending.clear();
        }
    }
    s.n_multi = (int64_t)me_end.size();
    s.n_zrows = G + s.n_multi;
    s.eblocks = (int)std::max<int64_t>(1, (s.n_multi + 255) / 256);
    s.ldz = std::max<int64_t>(128, (s.n_zrows + 127) / 128 * 128);   // K chunks of the contraction are 128 rows
    s.max_blocks = (int)((ld + 255) / 256) + 1;
    // column-pass tiles: the persistent kernel's tiles (ld = grid * tile)
    s.tile = ld / h->shape.grid;
    s.ntiles = h->shape.grid;
    std::vector<uint8_t> tile_carry(s.ntiles, 0);
    std::vector<int32_t> lasthead(s.ntiles, -1), agg_tiles;
    for (int t = 0; t < s.ntiles; ++t) {
        tile_carry[t] = head[(size_t)t * s.tile] ? 0 : 1;
        for (int64_t r = (int64_t)(t + 1) * s.tile - 1; r >= (int64_t)t * s.tile; --r)
            if (head[r]) {
                lasthead[t] = (int32_t)r;
                break;
            }
    }
    for (int t = 0; t + 1 < s.ntiles; ++t)
        if (tile_carry[t + 1]) agg_tiles.push_back(t);
    s.n_agg = (int)agg_tiles.size();
    s.syrk_part_bytes = lowp(h->opt.x_precision)
                            ? std::max({syrk_bf16_partial_bytes(p, 2 * kSplitsXBF16), syrk_bf16_partial_bytes(p, kSplitsXFP8),
                                        syrk_bf16_partial_bytes(p, 2 * kSplitsZBF16)})
                            : std::max(syrk_partial_bytes(p, (p <= 256 ? 2 : 1) * kSplitsXF64),
                                       syrk_partial_bytes(p, (p <= 256 ? 2 : 1) * kSplitsZF64));
    s.scan_scratch_bytes = rowscan_scratch_bytes(s.ntiles);
    const size_t zb = ztype_bytes(h->opt.x_precision);
    hipError_t e;
    if ((e = dalloc(&s.gidx, sizeof(int32_t) * ld)) != hipSuccess ||
        (e = dalloc(&s.rows, sizeof(double) * 9 * ld)) != hipSuccess ||
        (e = dalloc(&s.blockbuf, sizeof(double) * s.max_blocks)) != hipSuccess ||
        (e = dalloc(&s.tile_carry, (size_t)s.ntiles)) != hipSuccess ||
        (e = dalloc(&s.lasthead, sizeof(int32_t) * s.ntiles)) != hipSuccess ||
        (e = dalloc(&s.agg_tiles, sizeof(int32_t) * std::max(1, s.n_agg))) != hipSuccess ||
        (e = dalloc(&s.agg, sizeof(double) * 2 * (size_t)s.ntiles * p)) != hipSuccess ||
        (e = dalloc(&s.carry, sizeof(double) * (size_t)s.ntiles * p)) != hipSuccess ||
        (e = dalloc(&s.colpart, sizeof(double) * 3 * (size_t)s.ntiles * p)) != hipSuccess ||
        (e = dalloc(&s.vec, sizeof(double) * (5 * (size_t)p + kScalSlots))) != hipSuccess ||
        (e = dalloc(&s.flags, sizeof(unsigned))) != hipSuccess ||
        (e = dalloc(&s.status, sizeof(int))) != hipSuccess ||
        (e = dalloc(&s.free_col, (size_t)p)) != hipSuccess ||
        (e = dalloc(&s.z, zb * (size_t)p * s.ldz)) != hipSuccess ||
        (e = dalloc(&s.zscale, sizeof(float) * p)) != hipSuccess ||
        (e = dalloc(&s.syrk_part, s.syrk_part_bytes)) != hipSuccess ||
        (e = dalloc(&s.info, sizeof(double) * (size_t)p * p)) != hipSuccess ||
        (e = dalloc(&s.scan_scratch, s.scan_scratch_bytes)) != hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void **>(&s.hvec), sizeof(double) * (5 * (size_t)p + kScalSlots + 2),
                           hipHostMallocDefault)) != hipSuccess) {
        newton_free(h);
        return handle_hip_fail(h, e, "allocating full-evaluation buffers");
    }
    for (int k = 0; k < 6 && e == hipSuccess; ++k) e = hipEventCreate(&s.ev[k]);
    if (e != hipSuccess) {
        newton_free(h);
        return handle_hip_fail(h, e, "creating events");
    }
    e = hipMemcpy(s.gidx, gidx.data(), sizeof(int32_t) * ld, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s.tile_carry, tile_carry.data(), (size_t)s.ntiles, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(s.lasthead, lasthead.data(), sizeof(int32_t) * s.ntiles, hipMemcpyHostToDevice);
    if (e == hipSuccess && s.n_agg)
        e = hipMemcpy(s.agg_tiles, agg_tiles.data(), sizeof(int32_t) * s.n_agg, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(s.z, 0, zb * (size_t)p * s.ldz);
    if (e == hipSuccess && s.efron) {
        const size_t nme = std::max<size_t>(1, me_row.size()), nm = (size_t)std::max<int64_t>(1, s.n_multi);
        if (e == hipSuccess) e = dalloc(&s.gidx2, sizeof(int32_t) * ld);
        if (e == hipSuccess) e = dalloc(&s.gend, sizeof(int32_t) * ld);
        if (e == hipSuccess) e = dalloc(&s.me_ptr, sizeof(int32_t) * (nm + 1));
        if (e == hipSuccess) e = dalloc(&s.me_row, sizeof(int32_t) * nme);
        if (e == hipSuccess) e = dalloc(&s.me_end, sizeof(int32_t) * nm);
        if (e == hipSuccess) e = dalloc(&s.me_w, sizeof(double) * nme);
        if (e == hipSuccess) e = dalloc(&s.s1me, sizeof(double) * nm * p);
        if (e == hipSuccess) e = dalloc(&s.erows, sizeof(double) * 4 * ld);
        if (e == hipSuccess) e = dalloc(&s.epart, sizeof(double) * (size_t)s.eblocks * p);
        if (e == hipSuccess) e = hipMemcpy(s.gidx2, gidx2.data(), sizeof(int32_t) * ld, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s.gend, gend.data(), sizeof(int32_t) * ld, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(s.me_ptr, me_ptr.data(), sizeof(int32_t) * me_ptr.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && !me_row.empty())
            e = hipMemcpy(s.me_row, me_row.data(), sizeof(int32_t) * me_row.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && !me_end.empty())
            e = hipMemcpy(s.me_end, me_end.data(), sizeof(int32_t) * me_end.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(s.erows, 0, sizeof(double) * 4 * ld);
    }
    if (e != hipSuccess) {
        newton_free(h);
        return handle_hip_fail(h, e, "uploading group indices");
    }
    if (h->opt.x_precision == COX_FP8_E4M3) {
        // e4m3 copy of X with power-of-two column scales (|x / s| <= 224)
        if ((e = dalloc(&s.xlp, fp8_copy_bytes(ld, p))) != hipSuccess ||
            (e = dalloc(&s.xscale, sizeof(float) * p)) != hipSuccess ||
            (e = dalloc(&s.wscratch, sizeof(double) * 264)) != hipSuccess) {
            newton_free(h);
            return handle_hip_fail(h, e, "allocating the FP8 copy of X");
        }
        int rc = make_fp8_copy(h->d_x, ld, p, static_cast<uint8_t *>(s.xlp), s.xscale, s.zscale, h->stream);
        if (rc == 0 && hipStreamSynchronize(h->stream) != hipSuccess) rc = -3;
        if (rc != 0) {
            newton_free(h);
            return handle_fail(h, COX_EDEVICE, "building the FP8 copy of X");
        }
    }
    if (h->opt.x_precision == COX_BF16) {
        // low-precision copy of X with power-of-two column scales (|x / s| <= 1)
        if ((e = dalloc(&s.xlp, sizeof(uint16_t) * (size_t)p * ld)) != hipSuccess ||
            (e = dalloc(&s.xscale, sizeof(float) * p)) != hipSuccess) {
            newton_free(h);
            return handle_hip_fail(h, e, "allocating the BF16 copy of X");
        }
        int rc = make_bf16_copy(h->d_x, ld, p, s.xlp, s.xscale, s.zscale, h->stream);
        if (rc == 0 && hipStreamSynchronize(h->stream) != hipSuccess) rc = -3;
        if (rc != 0) {
            newton_free(h);
            return handle_fail(h, COX_EDEVICE, "building the BF16 copy of X");
        }
    }
    s.ready = true;
    return COX_OK;
}

struct EvalOut {
    double objective = 0.0;
    std::vector<double> grad, diag1, diag2;
    unsigned flags = 0;
};

// Full evaluation at beta (host); xbar (and diag2) only when want_xbar.
int newton_eval(cox_handle *h, const double *beta, bool want_xbar, EvalOut &out)
{
    NewtonState &s = h->nt;
    const int64_t ld = h->shape.ld;
    const int p = (int)h->p;
    double *d_beta = s.vec, *d_grad = s.vec + p, *d_d1 = s.vec + 2 * p, *d_d2 = s.vec + 3 * p;
    double *d_scal = s.vec + 5 * p;
    // beta goes up, and the results come back, through the pinned mirror: one
    // synchronisation per evaluation
    std::memcpy(s.hvec, beta, sizeof(double) * p);
    hipError_t e = hipMemcpyAsync(d_beta, s.hvec, sizeof(double) * p, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return handle_hip_fail(h, e, "staging beta");
    FullEvalArgs A;
    A.x = h->d_x;
    A.meta = h->d_meta;
    A.gidx = s.gidx;
    A.beta = d_beta;
    A.ld = ld;
    A.p = p;
    A.max_blocks = s.max_blocks;
    A.eta = nrow(s, ld, 0);
    A.w = nrow(s, ld, 1);
    A.s0 = nrow(s, ld, 2);
    A.h = nrow(s, ld, 3);
    A.lam = nrow(s, ld, 4);
    A.zq = nrow(s, ld, 7);
    A.m = nrow(s, ld, 8);
    A.alpha = nrow(s, ld, 5);
    A.b = nrow(s, ld, 6);
    A.blockbuf = s.blockbuf;
    A.tile = s.tile;
    A.ntiles = s.ntiles;
    A.tile_carry = s.tile_carry;
    A.lasthead = s.lasthead;
    A.agg_tiles = s.agg_tiles;
    A.n_agg = s.n_agg;
    A.agg = s.agg;
    A.carry = s.carry;
    A.colpart = s.colpart;
    A.grad = d_grad;
    A.diag1 = d_d1;
    A.diag2 = d_d2;
    A.scal = d_scal;
    A.flags = s.flags;
    A.ztype = lowp(h->opt.x_precision) ? kZBF16 : kZF64;
    A.z = s.z;
    A.ldz = s.ldz;
    A.zscale = lowp(h->opt.x_precision) ? s.zscale : nullptr;
    A.want_xbar = want_xbar;
    A.scan_scratch = s.scan_scratch;
    A.scan_scratch_bytes = s.scan_scratch_bytes;
    if (s.efron) {
        A.efron = true;
        A.e0 = s.erows;
        A.kq = s.erows + ld;
        A.zq2 = s.erows + 2 * ld;
        A.zq3 = s.erows + 3 * ld;
        A.gidx2 = s.gidx2;
        A.gend = s.gend;
        A.me_ptr = s.me_ptr;
        A.me_row = s.me_row;
        A.me_end = s.me_end;
        A.me_w = s.me_w;
        A.s1me = s.s1me;
        A.epart = s.epart;
        A.n_groups = s.n_groups;
        A.n_multi = s.n_multi;
        A.eblocks = s.eblocks;
    }
    (void)hipEventRecord(s.ev[0], h->stream);
    int rc = full_eval_launch(A, h->stream);
    if (rc != 0) return handle_fail(h, rc == -5 ? COX_EUNSUPPORTED : COX_EDEVICE, "full evaluation launch");
    (void)hipEventRecord(s.ev[1], h->stream);
    // grad, diag1, diag2, dx and scal are contiguous after beta
    double *hres = s.hvec + p;
    unsigned *hflags = reinterpret_cast<unsigned *>(s.hvec + 5 * p + kScalSlots);
    if ((e = hipMemcpyAsync(hres, d_grad, sizeof(double) * (4 * (size_t)p + kScalSlots), hipMemcpyDeviceToHost,
                            h->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(hflags, s.flags, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(h->stream)) != hipSuccess)
        return handle_hip_fail(h, e, "full evaluation");
    (void)d_d1;
    (void)d_d2;
    h->prof.evaluations += 1;
    h->prof.evaluation_ms += elapsed_ms(s.ev[0], s.ev[1]);
    out.grad.assign(hres, hres + p);
    out.diag1.assign(hres + p, hres + 2 * p);
    if (want_xbar) out.diag2.assign(hres + 2 * p, hres + 3 * p);
    else out.diag2.assign(p, 0.0);
    out.flags = *hflags;
    out.objective = hres[4 * p + 1];
    if (out.flags & 1u) return handle_fail(h, COX_ENUMERIC, "a risk-set sum left the FP64 normal range");
    return COX_OK;
}

// info = X' diag(b) X - Z'Z in the handle's precision, left in s.info (FP64).
int newton_info(cox_handle *h)
{
    NewtonState &s = h->nt;
    const int64_t ld = h->shape.ld;
    const int p = (int)h->p;
    const double *b = nrow(s, ld, 6);
    int rc;
    (void)hipEventRecord(s.ev[2], h->stream);
    if (lowp(h->opt.x_precision)) {
        if (h->opt.x_precision == COX_FP8_E4M3)
            rc = syrk_fp8(static_cast<const uint8_t *>(s.xlp), ld, p, s.xscale, b, ld, kSplitsXFP8, s.syrk_part,
                          s.wscratch, s.wscratch + 256, 1.0, 0, s.info, h->stream);
        else
            rc = syrk_bf16(static_cast<const uint16_t *>(s.xlp), ld, p, s.xscale, b, ld, kSplitsXBF16, s.syrk_part,
                           1.0, 0, s.info, h->stream);
        if (rc == 0 && s.n_zrows > 0)
            rc = syrk_bf16(static_cast<const uint16_t *>(s.z), s.ldz, p, s.zscale, nullptr, s.n_zrows, kSplitsZBF16,
                           s.syrk_part, -1.0, 1, s.info, h->stream);
    } else {
        rc = syrk_f64(h->d_x, ld, p, b, ld, kSplitsXF64, s.syrk_part, 1.0, 0, s.info, h->stream);
        if (rc == 0 && s.n_zrows > 0)
            rc = syrk_f64(static_cast<const double *>(s.z), s.ldz, p, nullptr, s.n_zrows, kSplitsZF64, s.syrk_part,
                          -1.0, 1, s.info, h->stream);
    }
    if (rc != 0) return handle_fail(h, COX_EDEVICE, "information-matrix contraction launch");
    (void)hipEventRecord(s.ev[3], h->stream);
    return COX_OK;
}

}  // namespace

void newton_free(cox_handle *h)
{
    NewtonState &s = h->nt;
    void *ptrs[] = {s.gidx, s.rows, s.blockbuf, s.tile_carry, s.lasthead, s.agg_tiles, s.agg, s.carry,
                    s.colpart, s.vec, s.flags, s.status, s.free_col, s.z,
                    s.zscale, s.xlp, s.xscale, s.syrk_part, s.info, s.scan_scratch, s.wscratch,
                    s.gidx2, s.gend, s.me_ptr, s.me_row, s.me_end, s.me_w, s.s1me, s.erows, s.epart, s.prox};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (s.hvec) (void)hipHostFree(s.hvec);
    for (hipEvent_t ev : s.ev)
        if (ev) (void)hipEventDestroy(ev);
    s = NewtonState();
}

extern "C" int cox_evaluate_full(cox_handle *h, const double *beta, double *objective, double *grad,
                                 double *hess_diag, double *info)
{
    if (!h) return handle_fail(nullptr, COX_EINVAL, "handle is NULL");
    if (!beta) return handle_fail(h, COX_EINVAL, "beta is NULL");
    (void)hipSetDevice(h->device);
    int rc = newton_setup(h);
    if (rc != COX_OK) return rc;
    h->prof = cox_profile{};
    EvalOut ev;
    rc = newton_eval(h, beta, hess_diag || info, ev);
    if (rc != COX_OK) return rc;
    const int p = (int)h->p;
    if (objective) {
        double pen = 0.0;
        for (int j = 0; j < p; ++j) pen += h->gamma[j] * std::fabs(beta[j]);
        *objective = ev.objective + pen;
    }
    if (grad) std::memcpy(grad, ev.grad.data(), sizeof(double) * p);
    if (hess_diag)
        for (int j = 0; j < p; ++j) hess_diag[j] = ev.diag1[j] - ev.diag2[j];
    if (info) {
        rc = newton_info(h);
        if (rc != COX_OK) return rc;
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e == hipSuccess)
            e = hipMemcpy(info, h->nt.info, sizeof(double) * (size_t)p * p, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return handle_hip_fail(h, e, "information matrix");
        h->prof.contractions += 1;
        h->prof.contraction_ms += elapsed_ms(h->nt.ev[2], h->nt.ev[3]);
    }
    return COX_OK;
}

extern "C" int cox_baseline_hazard(cox_handle *h, const double *beta, double *cumhaz)
{
    if (!h) return handle_fail(nullptr, COX_EINVAL, "handle is NULL");
    if (!beta || !cumhaz) return handle_fail(h, COX_EINVAL, "beta and cumhaz are required");
    if (h->opt.ties == COX_EFRON)
        return handle_fail(h, COX_EUNSUPPORTED, "the baseline hazard is the Breslow estimator (COX_BRESLOW handles)");
    (void)hipSetDevice(h->device);
    int rc = newton_setup(h);
    if (rc != COX_OK) return rc;
    EvalOut ev;
    rc = newton_eval(h, beta, false, ev);
    if (rc != COX_OK) return rc;
    // R_r = Lambda_r exp(m_r) (the reverse scan of the evaluation), m_r the running maximum of X beta
    const int64_t ld = h->shape.ld;
    std::vector<double> R((size_t)ld), m((size_t)ld);
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipMemcpy(R.data(), nrow(h->nt, ld, 4), sizeof(double) * ld, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(m.data(), nrow(h->nt, ld, 8), sizeof(double) * ld, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return handle_hip_fail(h, e, "reading the cumulative hazard");
    for (int64_t c = 0; c < h->n; ++c) {
        const int64_t r = h->pos[(size_t)c];
        cumhaz[h->perm[(size_t)c]] = R[(size_t)r] * std::exp(-m[(size_t)r]);
    }
    return COX_OK;
}

// Proximal Newton for the l1-penalised fit: each step minimises the quadratic model
//   g'D + D'HD/2 + sum_j gamma_j |beta_j + D_j|
// (FP64 score g, information H in x_precision) by cyclic coordinate descent with soft
// thresholding on the device (prox_model_solve: H stays where the contraction left it; only
// g, beta and D cross to and from the host); a step that raises the penalised objective is halved.  A fixed
// point (D = 0) satisfies the l1 optimality conditions on the FP64 score whatever the
// precision of H, so a reduced-precision H, kept once steps are small, still reaches the
// FP64 optimum.
static int newton_fit_l1(cox_handle *h, const double *beta0, double *beta_out, cox_fit_info *info)
{
    NewtonState &s = h->nt;
    const int p = (int)h->p;
    const std::vector<double> &gam = h->gamma;
    std::vector<double> beta(p, 0.0), prev(p, 0.0), D(p, 0.0);
    if (!s.prox) {
        const hipError_t e = hipMalloc(&s.prox, sizeof(double) * (4 * (size_t)p + 1));
        if (e != hipSuccess) {
            s.prox = nullptr;
            return handle_hip_fail(h, e, "proximal Newton buffers");
        }
    }
    double *d_g = s.prox, *d_beta = s.prox + p, *d_gam = s.prox + 2 * p, *d_D = s.prox + 3 * p;
    int *d_sweeps = reinterpret_cast<int *>(s.prox + 4 * p);
    {
        const hipError_t e = hipMemcpy(d_gam, gam.data(), sizeof(double) * p, hipMemcpyHostToDevice);
        if (e != hipSuccess) return handle_hip_fail(h, e, "l1 weights");
    }
    if (beta0) std::memcpy(beta.data(), beta0, sizeof(double) * p);
    std::vector<uint8_t> freec(p, 1);
    bool frozen = false, have_free = false, have_h = false, converged = false;
    double obj_prev = INFINITY, last_step = 0.0, objective = 0.0;
    int iters = 0, evals = 0, halvings = 0;
    auto penalty = [&](const std::vector<double> &b) {
        double v = 0.0;
        for (int j = 0; j < p; ++j) v += gam[j] * std::fabs(b[j]);
        return v;
    };
    EvalOut ev;
    while (iters < h->opt.max_iter) {
        int rc = newton_eval(h, beta.data(), !frozen || !have_free, ev);
        ++evals;
        if (rc != COX_OK) return rc;
        if (!have_free) {
            bool moved = false;
            for (int j = 0; j < p; ++j) {
                const double hd = ev.diag1[j] - ev.diag2[j];
                freec[j] = (hd > 1e-12 * std::fabs(ev.diag1[j]) && std::isfinite(hd)) ? 1 : 0;
                if (!freec[j] && beta[j] != 0.0) {
                    beta[j] = 0.0;
                    moved = true;
                }
            }
            have_free = true;
            const hipError_t e = hipMemcpy(s.free_col, freec.data(), (size_t)p, hipMemcpyHostToDevice);
            if (e != hipSuccess) return handle_hip_fail(h, e, "free columns");
            if (moved) continue;   // re-evaluate at the start point with the pinned columns at zero
        }
        const double F = ev.objective + penalty(beta);
        if (F > obj_prev + 1e-12 * std::fabs(obj_prev) && halvings < 40) {
            for (int j = 0; j < p; ++j) beta[j] = prev[j] + 0.5 * (beta[j] - prev[j]);
            ++halvings;
            continue;
        }
        halvings = 0;
        objective = F;
        if (!frozen || !have_h) {
            rc = newton_info(h);
            if (rc != COX_OK) return rc;
            const hipError_t e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) return handle_hip_fail(h, e, "information matrix");
            h->prof.contractions += 1;
            h->prof.contraction_ms += elapsed_ms(s.ev[2], s.ev[3]);
            have_h = true;
        }
        // coordinate descent on the model (device).  The model is solved to a thousandth of the
        // last outer step (inexact early on), and to 1e-3 tol at the end
        double bmax = 1.0;
        for (int j = 0; j < p; ++j) bmax = std::max(bmax, std::fabs(beta[j]));
        const double inner_tol = std::max(1e-3 * h->opt.tol * bmax, iters ? 1e-3 * last_step : 1e-3 * bmax);
        {
            hipError_t e = hipMemcpyAsync(d_g, ev.grad.data(), sizeof(double) * p, hipMemcpyHostToDevice, h->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d_beta, beta.data(), sizeof(double) * p, hipMemcpyHostToDevice, h->stream);
            if (e == hipSuccess) e = hipEventRecord(s.ev[4], h->stream);
            if (e == hipSuccess &&
                prox_model_solve(s.info, p, d_g, d_beta, d_gam, s.free_col, inner_tol, 1000, d_D, d_sweeps,
                                 h->stream) != 0)
                e = hipErrorLaunchFailure;
            if (e == hipSuccess) e = hipEventRecord(s.ev[5], h->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(D.data(), d_D, sizeof(double) * p, hipMemcpyDeviceToHost, h->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) return handle_hip_fail(h, e, "proximal model solve");
            h->prof.solves += 1;
            h->prof.solve_ms += elapsed_ms(s.ev[4], s.ev[5]);
        }
        prev = beta;
        obj_prev = F;
        double step = 0.0;
        for (int j = 0; j < p; ++j) {
            const double nb = beta[j] + D[j];   // exactly 0 where the model's soft threshold gave 0
            beta[j] = nb == 0.0 ? 0.0 : nb;
            step = std::max(step, std::fabs(D[j]));
        }
        bmax = 1.0;
        for (int j = 0; j < p; ++j) bmax = std::max(bmax, std::fabs(beta[j]));
        ++iters;
        last_step = step;
        if (step <= h->opt.tol * bmax) {
            converged = true;
            break;
        }
        if (!frozen && h->opt.x_precision != COX_F64 && step <= 1e-3 * bmax) frozen = true;
    }
    std::memcpy(beta_out, beta.data(), sizeof(double) * p);
    const int rc = converged ? COX_OK : COX_NOT_CONVERGED;
    if (info) {
        info->status = rc;
        info->iters = iters;
        info->coord_evals = evals;
        info->objective = objective;
        info->last_step = last_step;
        int pinned = 0;
        double kkt = 0.0;
        for (int j = 0; j < p; ++j) {
            if (!freec[j]) {
                ++pinned;
                continue;
            }
            const double g = ev.grad[j], b = beta_out[j];
            const double r = gam[j] <= 0.0 ? std::fabs(g)
                                           : (b != 0.0 ? std::fabs(g + (b > 0 ? gam[j] : -gam[j]))
                                                       : std::max(std::fabs(g) - gam[j], 0.0));
            kkt = std::max(kkt, r);
        }
        info->n_pinned = pinned;
        info->kkt_inf = kkt;
    }
    return rc;
}

int newton_fit(cox_handle *h, const double *beta0, double *beta_out, cox_fit_info *info)
{
    {
        bool penalised = false;
        for (double g : h->gamma) penalised = penalised || g != 0.0;
        if (penalised) {
            (void)hipSetDevice(h->device);
            const int rc0 = newton_setup(h);
            if (rc0 != COX_OK) return rc0;
            h->prof = cox_profile{};
            return newton_fit_l1(h, beta0, beta_out, info);
        }
    }
    (void)hipSetDevice(h->device);
    int rc = newton_setup(h);
    if (rc != COX_OK) return rc;
    NewtonState &s = h->nt;
    const int p = (int)h->p;
    h->prof = cox_profile{};
    std::vector<double> beta(p, 0.0), prev(p, 0.0), dx(p, 0.0);
    if (beta0) std::memcpy(beta.data(), beta0, sizeof(double) * p);
    std::vector<uint8_t> freec(p, 1);
    double *d_grad = s.vec + p, *d_dx = s.vec + 4 * p;
    bool frozen = false, have_free = false, converged = false;
    double obj_prev = INFINITY, last_step = 0.0, objective = 0.0;
    int iters = 0, evals = 0, halvings = 0;
    EvalOut ev;
    while (iters < h->opt.max_iter) {
        rc = newton_eval(h, beta.data(), !frozen || !have_free, ev);
        ++evals;
        if (rc != COX_OK) return rc;
        if (!have_free) {
            for (int j = 0; j < p; ++j) {
                const double hd = ev.diag1[j] - ev.diag2[j];
                freec[j] = (hd > 1e-12 * std::fabs(ev.diag1[j]) && std::isfinite(hd)) ? 1 : 0;
            }
            hipError_t e = hipMemcpy(s.free_col, freec.data(), (size_t)p, hipMemcpyHostToDevice);
            if (e != hipSuccess) return handle_hip_fail(h, e, "free columns");
            have_free = true;
        }
        // a step that raised the objective is halved (and re-evaluated)
        if (ev.objective > obj_prev + 1e-12 * std::fabs(obj_prev) && halvings < 40) {
            for (int j = 0; j < p; ++j) beta[j] = prev[j] + 0.5 * (beta[j] - prev[j]);
            ++halvings;
            continue;
        }
        halvings = 0;
        objective = ev.objective;
        if (!frozen) {
            rc = newton_info(h);
            if (rc != COX_OK) return rc;
        }
        (void)hipEventRecord(s.ev[4], h->stream);
        if (chol_solve(s.info, p, d_grad, s.free_col, frozen ? 1 : 0, d_dx, s.status, h->stream) != 0)
            return handle_fail(h, COX_EDEVICE, "Cholesky launch");
        (void)hipEventRecord(s.ev[5], h->stream);
        int *hstatus = reinterpret_cast<int *>(s.hvec + 5 * p + kScalSlots + 1);
        double *hdx = s.hvec + 4 * p;
        hipError_t e = hipMemcpyAsync(hdx, d_dx, sizeof(double) * p, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(hstatus, s.status, sizeof(int), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (!frozen) {
            h->prof.contractions += 1;
            h->prof.contraction_ms += elapsed_ms(s.ev[2], s.ev[3]);
        }
        h->prof.solves += 1;
        h->prof.solve_ms += elapsed_ms(s.ev[4], s.ev[5]);
        if (e != hipSuccess) return handle_hip_fail(h, e, "Cholesky solve");
        const int status = *hstatus;
        std::memcpy(dx.data(), hdx, sizeof(double) * p);
        if (status) return handle_fail(h, COX_ENUMERIC, "the information matrix is not positive definite");
        prev = beta;
        obj_prev = ev.objective;
        double step = 0.0, bmax = 1.0;
        for (int j = 0; j < p; ++j) {
            beta[j] += dx[j];
            step = std::max(step, std::fabs(dx[j]));
        }
        for (int j = 0; j < p; ++j) bmax = std::max(bmax, std::fabs(beta[j]));
        ++iters;
        last_step = step;
        if (step <= h->opt.tol * bmax) {
            converged = true;
            break;
        }
        if (!frozen && h->opt.x_precision != COX_F64 && step <= 1e-3 * bmax) frozen = true;
    }
    std::memcpy(beta_out, beta.data(), sizeof(double) * p);
    rc = converged ? COX_OK : COX_NOT_CONVERGED;
    if (info) {
        info->status = rc;
        info->iters = iters;
        info->coord_evals = evals;
        info->objective = objective;
        info->last_step = last_step;
        int pinned = 0;
        double kkt = 0.0;
        for (int j = 0; j < p; ++j) {
            if (!freec[j]) ++pinned;
            else kkt = std::max(kkt, std::fabs(ev.grad[j]));
        }
        info->n_pinned = pinned;
        info->kkt_inf = kkt;
    }
    return rc;
}
