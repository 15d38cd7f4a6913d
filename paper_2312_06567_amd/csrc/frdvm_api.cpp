// Compute entry points of the C ABI (include/fr_dvm.h): orchestration of the
// moment, Newton, FR-stage and collision kernels on the handle's stream.
#include <hip/hip_runtime.h>

#include <cstring>
#include <utility>

#include "../../include/fr_dvm_mlp.h"
#include "frdvm_common.h"

using namespace frdvm;

namespace {

int ready(fr_dvm *h) {
    if (!h) return FR_DVM_EINVAL;
    if (!h->have_params) return h->fail(FR_DVM_EINVAL, "fr_dvm_set_params has not been called");
    return FR_DVM_OK;
}

StageArgs blank() {
    StageArgs a;
    std::memset(&a, 0, sizeof(a));
    a.beta = 1.0;
    return a;
}

// Moments (and, if traces, the outflow traces) of f into h->d_Q / h->d_tr[cur].
int prime(fr_dvm *h, const void *f, int traces, int moments) {
    StageArgs a = blank();
    a.f = f;
    a.tr_out = h->d_tr[h->cur_tr];
    a.Q = h->d_Q;
    ProfScope ps(h, 2);
    return launch_fr(h, 0, a, traces, moments);
}

int guess_mode(fr_dvm *h) {
    if (h->prm.guess == FR_DVM_GUESS_MLP && !h->d_mlp) return FR_DVM_GUESS_COLD;
    return h->prm.guess;
}

}  // namespace

extern "C" int fr_dvm_moments(fr_dvm_t h, const void *f, double *Q, double *totals) {
    int rc = ready(h);
    if (rc) return rc;
    if (!f) return h->fail(FR_DVM_EINVAL, "null f");
    if ((rc = prime(h, f, 0, 1))) return rc;
    if (Q && (rc = launch_moments_out(h, Q))) return rc;
    if (totals && (rc = launch_totals(h, totals))) return rc;
    return FR_DVM_OK;
}

extern "C" int fr_dvm_kn_gll(fr_dvm_t h, const void *f, double *kn) {
    int rc = ready(h);
    if (rc) return rc;
    if (!f || !kn) return h->fail(FR_DVM_EINVAL, "null f or kn");
    if (h->mx) return h->fail(FR_DVM_EUNSUPPORTED, "the Knudsen-number field needs a hexahedral mesh");
    if ((rc = prime(h, f, 0, 1))) return rc;
    return launch_kn_gll(h, kn);
}

extern "C" int fr_dvm_residual(fr_dvm_t h, const void *f, void *R) {
    int rc = ready(h);
    if (rc) return rc;
    if (!f || !R) return h->fail(FR_DVM_EINVAL, "null f or R");
    if (f == R) return h->fail(FR_DVM_EINVAL, "R must not alias f");
    if ((rc = prime(h, f, 1, 0))) return rc;
    StageArgs a = blank();
    a.f = f;
    a.fout = R;
    a.tr_in = h->d_tr[h->cur_tr];
    return launch_fr(h, 2, a, 0, 0);
}

extern "C" int fr_dvm_collide(fr_dvm_t h, const void *f, void *S, double *Qp, int accumulate) {
    int rc = ready(h);
    if (rc) return rc;
    if (!f || !S) return h->fail(FR_DVM_EINVAL, "null f or S");
    if (h->prm.model == FR_DVM_FREE) {
        if (!accumulate) {
            size_t es = h->prm.precision == FR_DVM_FP64 ? sizeof(double) : sizeof(float);
            if (hipMemsetAsync(S, 0, es * h->ne * h->ns * h->vg.nu * h->ncomp, h->stream) != hipSuccess)
                return h->fail(FR_DVM_EHIP, "memset");
        }
        if (Qp && hipMemsetAsync(Qp, 0, sizeof(double) * 5 * h->ne * h->ns, h->stream) != hipSuccess)
            return h->fail(FR_DVM_EHIP, "memset");
        return FR_DVM_OK;
    }
    if ((rc = prime(h, f, 0, 1))) return rc;
    if ((rc = launch_newton(h, guess_mode(h)))) return rc;
    if ((rc = launch_collide(h, f, S, accumulate))) return rc;
    if (Qp && (rc = launch_prim_out(h, Qp))) return rc;
    return FR_DVM_OK;
}

namespace {

// Arguments of RK stage st (0..2) of the handle's scheme, f updated in place.
StageArgs stage_args(fr_dvm *h, void *f, double dt, int st, int collide) {
    StageArgs a = blank();
    a.dt = dt;
    a.collide = collide;
    a.positivity = h->prm.positivity;
    a.seed = (h->stage_count++) * 0x9e3779b9u;  // a different seed for every stage
    a.eq = h->d_eq;
    a.tr_in = h->d_tr[h->cur_tr];
    a.tr_out = h->d_tr[h->cur_tr ^ 1];
    a.Q = h->d_Q;
    if (h->prm.rk == FR_DVM_SSPRK3) {
        static const double al[3] = {0.0, 0.75, 1.0 / 3.0}, be[3] = {1.0, 0.25, 2.0 / 3.0};
        a.scheme = 0;
        a.alpha = al[st];
        a.beta = be[st];
        a.f = st == 0 ? f : h->d_reg;
        a.fn = f;
        a.fout = st == 2 ? f : h->d_reg;
    } else {
        static const double lA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0}, lB[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
        a.scheme = 1;
        a.lsA = lA[st];
        a.lsB = lB[st];
        a.keep_dF = st < 2;
        a.f = f;
        a.fout = f;
        a.dF = h->d_reg;
    }
    return a;
}

// element references of the records just solved, into the current set
int elem_ref(fr_dvm *h) {
    ProfScope ps(h, 3);
    return launch_elem_ref(h, h->d_ref[h->cur_ref]);
}

int ensure_aux(fr_dvm *h) {
    if (h->aux) return FR_DVM_OK;
    if (hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) != hipSuccess) {
        h->aux = nullptr;
        return h->fail(FR_DVM_EHIP, "second stream");
    }
    for (int i = 0; i < 2; ++i)
        if (hipEventCreateWithFlags(&h->ev_stage[i], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&h->ev_newton[i], hipEventDisableTiming) != hipSuccess)
            return h->fail(FR_DVM_EHIP, "stream events");
    return FR_DVM_OK;
}

}  // namespace

extern "C" int fr_dvm_rk_steps(fr_dvm_t h, void *f, double dt, int nsteps) {
    int rc = ready(h);
    if (rc) return rc;
    if (!f) return h->fail(FR_DVM_EINVAL, "null f");
    if (nsteps < 0) return h->fail(FR_DVM_EINVAL, "nsteps < 0");
    if (nsteps == 0) return FR_DVM_OK;
    const int collide = h->prm.model != FR_DVM_FREE;
    // traces and moments of the incoming f (afterwards each stage leaves those
    // of its result for the next stage)
    if ((rc = prime(h, f, 1, collide))) return rc;
    const int guess = guess_mode(h);
    if (collide && (rc = launch_newton(h, guess))) return rc;
    // Overlap: the elements are taken in two halves (z slabs).  Stage k of
    // half 0, then of half 1, on the handle's stream; as soon as stage k of a
    // half is done, the Newton solve for stage k+1 of that half runs on the
    // second stream, alongside the stage launch of the other half.  Stage k+1
    // of a half waits for that half's Newton; it follows stage k of both
    // halves on its own stream (the neighbour traces it reads).  Per point
    // the work and its order are those of the single-stream path.
    // (decided after the first solve: a learned-then-warm start is warm from here on)
    // FP32 deviation storage: each stage reads its value relative to the
    // element references of the previous stage's records and writes relative
    // to those of its own (SSP also reads the step's initial value, relative
    // to the references it was written with): each stage's references go to
    // a set that neither of the others it reads holds; the first stage reads
    // plain f and takes its own references for both
    const bool dev = h->prm.precision == FR_DVM_FP32_DEV && collide;
    const bool ssp = h->prm.rk == FR_DVM_SSPRK3;
    if (dev) {
        h->cur_ref = h->prev_ref = h->u0_ref = 0;
        if ((rc = elem_ref(h))) return rc;
    }
    bool fn_dev = false;  // (SSP) f holds the step's initial value as deviations
    const bool split = h->prm.overlap && h->axis_mode && collide && !dev && h->ne >= 2 && newton_part_ok(h, guess);
    if (split && (rc = ensure_aux(h))) return rc;
    const int64_t eh[3] = {0, h->ne / 2, h->ne};
    const int nst = 3 * nsteps;
    for (int k = 0; k < nst; ++k) {
        const int st = k % 3;
        const int last = k == nst - 1;
        const int traces = last ? 0 : 1, moments = (last || !collide) ? 0 : 1;
        if (!split && k > 0 && collide) {
            if ((rc = launch_newton(h, guess))) return rc;
            if (dev) {
                h->prev_ref = h->cur_ref;
                int c = 0;
                while (c == h->prev_ref || (ssp && fn_dev && c == h->u0_ref)) ++c;
                h->cur_ref = c;
                if ((rc = elem_ref(h))) return rc;
            }
        }
        StageArgs a = stage_args(h, f, dt, st, collide);
        a.in_dev = dev && k > 0;
        a.out_dev = dev && !last;
        a.fn_dev = dev && fn_dev;
        a.ref_cur = h->d_ref[h->cur_ref];
        a.ref_prev = h->d_ref[h->prev_ref];
        a.ref_u0 = h->d_ref[h->u0_ref];
        if (!split) {
            ProfScope ps(h, 0);
            if ((rc = launch_fr(h, 1, a, traces, moments))) return rc;
        } else {
            for (int half = 0; half < 2; ++half) {
                if (k > 0 && hipStreamWaitEvent(h->stream, h->ev_newton[half], 0) != hipSuccess)
                    return h->fail(FR_DVM_EHIP, "stream wait");
                a.e0 = eh[half];
                a.ecount = eh[half + 1] - eh[half];
                {
                    ProfScope ps(h, 0);
                    if ((rc = launch_fr(h, 1, a, traces, moments))) return rc;
                }
                if (last) continue;
                if (hipEventRecord(h->ev_stage[half], h->stream) != hipSuccess ||
                    hipStreamWaitEvent(h->aux, h->ev_stage[half], 0) != hipSuccess)
                    return h->fail(FR_DVM_EHIP, "stream event");
                if ((rc = launch_newton_part(h, guess, eh[half] * h->ns, (eh[half + 1] - eh[half]) * h->ns, h->aux)))
                    return rc;
                if (hipEventRecord(h->ev_newton[half], h->aux) != hipSuccess)
                    return h->fail(FR_DVM_EHIP, "stream event");
            }
        }
        h->cur_tr ^= 1;
        // the result of a step's last stage is the next step's initial value
        if (dev && st == 2) {
            fn_dev = !last;
            h->u0_ref = h->cur_ref;
        }
    }
    return FR_DVM_OK;
}

extern "C" int fr_dvm_rk_step(fr_dvm_t h, void *f, double dt) { return fr_dvm_rk_steps(h, f, dt, 1); }

extern "C" int fr_dvm_newton_stats(fr_dvm_t h, int64_t *iters_hist, int64_t *n_fallback, int64_t *n_guard,
                                   int64_t *n_evals, double *max_resid, int reset) {
    if (!h) return FR_DVM_EINVAL;
    int64_t buf[kHist + 4];
    double mr;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return h->fail(FR_DVM_EHIP, "stream synchronise");
    if (hipMemcpy(buf, h->d_stats, sizeof(buf), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(&mr, h->d_maxres, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return h->fail(FR_DVM_EHIP, "stats copy");
    if (iters_hist) std::memcpy(iters_hist, buf, kHist * sizeof(int64_t));
    if (n_fallback) *n_fallback = buf[kHist];
    if (n_guard) *n_guard = buf[kHist + 1];
    if (n_evals) *n_evals = buf[kHist + 2];
    if (max_resid) *max_resid = mr;
    if (reset) {
        hipMemset(h->d_stats, 0, sizeof(buf));
        hipMemset(h->d_maxres, 0, sizeof(double));
    }
    return FR_DVM_OK;
}

extern "C" int fr_dvm_newton_points(fr_dvm_t h, int32_t *status, int32_t *iters, double *resid) {
    int rc = ready(h);
    if (rc) return rc;
    if (!h->newton_done) return h->fail(FR_DVM_EINVAL, "no conservative-equilibrium solve has run yet");
    const size_t n = (size_t)h->ne * h->ns;
    if ((status && hipMemcpyAsync(status, h->d_pt_status, n * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream) !=
                       hipSuccess) ||
        (iters && hipMemcpyAsync(iters, h->d_pt_iters, n * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream) !=
                      hipSuccess) ||
        (resid && hipMemcpyAsync(resid, h->d_pt_resid, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream) !=
                      hipSuccess))
        return h->fail(FR_DVM_EHIP, "per-point Newton outcome copy");
    return FR_DVM_OK;
}

extern "C" int fr_dvm_mlp_set_weights(fr_dvm_t h, const float *w, size_t n) {
    if (!h || !w) return FR_DVM_EINVAL;
    // FR_MLP_INPUTS -> H -> H -> H -> 5 plus 10 output affine floats: solve for H
    int H = 0;
    for (int c = 1; c <= 64; ++c) {
        if (fr_mlp_param_count(c) == n) { H = c; break; }
    }
    if (!H) return h->fail(FR_DVM_EINVAL, "weight count does not match a network of fr_mlp_param_count(H), H <= 64");
    if (h->d_mlp) { hipFree(h->d_mlp); h->d_mlp = nullptr; h->owned_bytes -= h->mlp_n * sizeof(float); }
    if (hipMalloc(&h->d_mlp, n * sizeof(float)) != hipSuccess) { h->d_mlp = nullptr; return h->fail(FR_DVM_ENOMEM, "mlp"); }
    h->owned_bytes += n * sizeof(float);
    if (hipMemcpy(h->d_mlp, w, n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return h->fail(FR_DVM_EHIP, "mlp upload");
    h->mlp_n = n;
    h->mlp_hidden = H;
    return FR_DVM_OK;
}

extern "C" int fr_dvm_profile(fr_dvm_t h, int enable) {
    if (!h) return FR_DVM_EINVAL;
    h->prof = enable != 0;
    return FR_DVM_OK;
}

extern "C" int fr_dvm_profile_read(fr_dvm_t h, double *ms, int64_t *launches, int reset) {
    if (!h) return FR_DVM_EINVAL;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return h->fail(FR_DVM_EHIP, "stream synchronise");
    for (auto &r : h->prof_recs) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
            h->prof_ms[r.kind] += t;
            h->prof_n[r.kind] += 1;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    h->prof_recs.clear();
    for (int k = 0; k < FR_DVM_PROF_KINDS; ++k) {
        if (ms) ms[k] = h->prof_ms[k];
        if (launches) launches[k] = h->prof_n[k];
        if (reset) { h->prof_ms[k] = 0; h->prof_n[k] = 0; }
    }
    return FR_DVM_OK;
}

extern "C" int fr_dvm_equilibrium(fr_dvm_t h, const double *Q, int64_t n, int guess, double *z, int32_t *iters,
                                  int32_t *evals, int32_t *status, double *resid) {
    int rc = ready(h);
    if (rc) return rc;
    if (n < 0 || (n > 0 && !Q)) return h->fail(FR_DVM_EINVAL, "bad moment array");
    if (guess != FR_DVM_GUESS_COLD && guess != FR_DVM_GUESS_MLP) return h->fail(FR_DVM_EINVAL, "guess must be cold or MLP");
    return launch_newton_points(h, Q, n, guess, z, iters, evals, status, resid);
}
