// C ABI entry points (include/tnmh.h): argument checks, ownership of device
// buffers, dispatch to the kernels.  No exception crosses the boundary.
#include "common.hpp"

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

int tn_fail(tn_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int tn_ensure(tn_ctx *ctx, void **ptr, size_t *cap, size_t bytes) {
    if (bytes <= *cap && *ptr) return TN_OK;
    if (*ptr) {
        TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
        TN_HIP(ctx, hipFree(*ptr));
        *ptr = nullptr;
        *cap = 0;
    }
    if (bytes == 0) bytes = 256;
    if (hipMalloc(ptr, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
        return tn_fail(ctx, TN_ENOMEM, "device allocation of " + std::to_string(bytes) +
                                           " bytes failed");
    }
    *cap = bytes;
    return TN_OK;
}

namespace {

void free_all(tn_ctx *ctx) {
    void *bufs[] = {ctx->Jh,    ctx->Jv,   ctx->h,    ctx->env,  ctx->dims,   ctx->ell,
                    ctx->G64r,  ctx->G32R, ctx->G16R, ctx->fac,  ctx->xbox,   ctx->wbuf,
                    ctx->scal,  ctx->xdims, ctx->gscr, ctx->pspins, ctx->counters,
                    ctx->cst,   ctx->gradscr};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
}

int check_prec(tn_ctx *ctx, int prec) {
    if (prec != TN_FP64 && prec != TN_FP32 && prec != TN_BF16)
        return tn_fail(ctx, TN_EINVAL, "prec must be TN_FP64, TN_FP32 or TN_BF16");
    return TN_OK;
}

// Copy the couplings into context-owned buffers and record the instance.
int set_instance(tn_ctx *ctx, int Lx, int Ly, const double *Jh, const double *Jv,
                 const double *h, double beta, int D, int prec) {
    if (Lx < 1 || Ly < 1) return tn_fail(ctx, TN_EINVAL, "Lx and Ly must be >= 1");
    if (Lx > 256) return tn_fail(ctx, TN_EINVAL, "Lx above 256 is not supported");
    if (D < 1 || D > TN_MAX_D) return tn_fail(ctx, TN_EINVAL, "D must be in 1..64");
    if (!std::isfinite(beta)) return tn_fail(ctx, TN_EINVAL, "beta must be finite");
    if (Lx > 1 && !Jh) return tn_fail(ctx, TN_EINVAL, "Jh is NULL");
    if (Ly > 1 && !Jv) return tn_fail(ctx, TN_EINVAL, "Jv is NULL");
    int rc;
    if ((rc = check_prec(ctx, prec))) return rc;
    const size_t nh = (size_t)Ly * (Lx - 1), nv = (size_t)(Ly - 1) * Lx, nf = (size_t)Ly * Lx;
    if (ctx->Jh) (void)hipFree(ctx->Jh);
    if (ctx->Jv) (void)hipFree(ctx->Jv);
    if (ctx->h) (void)hipFree(ctx->h);
    ctx->Jh = ctx->Jv = ctx->h = nullptr;
    TN_HIP(ctx, hipMalloc((void **)&ctx->Jh, (nh ? nh : 1) * sizeof(double)));
    TN_HIP(ctx, hipMalloc((void **)&ctx->Jv, (nv ? nv : 1) * sizeof(double)));
    if (nh)
        TN_HIP(ctx, hipMemcpyAsync(ctx->Jh, Jh, nh * sizeof(double), hipMemcpyDefault, ctx->stream));
    if (nv)
        TN_HIP(ctx, hipMemcpyAsync(ctx->Jv, Jv, nv * sizeof(double), hipMemcpyDefault, ctx->stream));
    if (h) {
        TN_HIP(ctx, hipMalloc((void **)&ctx->h, nf * sizeof(double)));
        TN_HIP(ctx, hipMemcpyAsync(ctx->h, h, nf * sizeof(double), hipMemcpyDefault, ctx->stream));
    }
    ctx->Lx = Lx;
    ctx->Ly = Ly;
    ctx->D = D;
    ctx->Dp = ((D + 15) / 16) * 16;
    ctx->beta = beta;
    ctx->prec = prec;
    ctx->has_env = false;
    const size_t envn = (size_t)(Ly + 1) * Lx * 2 * D * D;
    if ((rc = tn_ensure(ctx, (void **)&ctx->env, &ctx->env_cap, envn * sizeof(double)))) return rc;
    if (ctx->dims) (void)hipFree(ctx->dims);
    if (ctx->ell) (void)hipFree(ctx->ell);
    if (ctx->cst) (void)hipFree(ctx->cst);
    ctx->dims = nullptr;
    ctx->ell = nullptr;
    ctx->cst = nullptr;
    ctx->has_cst = false;
    TN_HIP(ctx, hipMalloc((void **)&ctx->dims, (size_t)(Ly + 1) * (Lx + 1) * sizeof(int)));
    TN_HIP(ctx, hipMalloc((void **)&ctx->ell, (size_t)(Ly + 1) * sizeof(double)));
    TN_HIP(ctx, hipMalloc((void **)&ctx->cst, (size_t)(Ly + 1) * sizeof(int)));
    TN_HIP(ctx, hipMemsetAsync(ctx->cst, 0xff, (size_t)(Ly + 1) * sizeof(int), ctx->stream));
    TN_HIP(ctx, hipMemsetAsync(ctx->ell, 0, (size_t)(Ly + 1) * sizeof(double), ctx->stream));
    return TN_OK;
}

int need_env(tn_ctx *ctx) {
    if (!ctx) return TN_EINVAL;
    if (!ctx->has_env) return tn_fail(ctx, TN_ESTATE, "no environment: call tn_build_env first");
    return TN_OK;
}

}  // namespace

extern "C" {

int tn_create(tn_ctx **out, void *hip_stream) {
    if (!out) return TN_EINVAL;
    *out = nullptr;
    tn_ctx *ctx = new (std::nothrow) tn_ctx();
    if (!ctx) return TN_ENOMEM;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&ctx->device) != hipSuccess ||
        hipMalloc((void **)&ctx->counters, CNT_N * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void **)&ctx->scal, 16 * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&ctx->xdims, 4096 * sizeof(int)) != hipSuccess ||
        hipMemset(ctx->counters, 0, CNT_N * sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        free_all(ctx);
        delete ctx;
        return TN_EHIP;
    }
    *out = ctx;
    return TN_OK;
}

int tn_destroy(tn_ctx *ctx) {
    if (!ctx) return TN_OK;
    (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
    return TN_OK;
}

const char *tn_last_error(const tn_ctx *ctx) {
    return ctx ? ctx->err.c_str() : "NULL context";
}

int tn_build_env(tn_ctx *ctx, int Lx, int Ly, const double *Jh, const double *Jv,
                 const double *h, double beta, int D, int prec, double *logZ_out) {
    (void)hipGetLastError();
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    int rc;
    if ((rc = set_instance(ctx, Lx, Ly, Jh, Jv, h, beta, D, prec))) return rc;
    double lz = 0.0;
    if ((rc = tn_env_build_device(ctx, &lz))) return rc;
    if ((rc = tn_make_operands(ctx, prec))) return rc;
    ctx->has_env = true;
    ctx->has_cst = true;
    if (logZ_out) {
        TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
        *logZ_out = lz;
    }
    return TN_OK;
}

int tn_set_env(tn_ctx *ctx, int Lx, int Ly, const double *Jh, const double *Jv,
               const double *h, double beta, int D, int prec, const double *env,
               const int *dims, const double *ell, double logZ) {
    (void)hipGetLastError();
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    if (Ly > 1 && (!env || !dims)) return tn_fail(ctx, TN_EINVAL, "env or dims is NULL");
    int rc;
    if ((rc = set_instance(ctx, Lx, Ly, Jh, Jv, h, beta, D, prec))) return rc;
    const size_t box = (size_t)2 * D * D;
    if (Ly > 1) {
        for (int k = 1; k < Ly; ++k)
            for (int c = 0; c <= Lx; ++c) {
                const int d = dims[(size_t)(k - 1) * (Lx + 1) + c];
                if (d < 1 || d > D || ((c == 0 || c == Lx) && d != 1))
                    return tn_fail(ctx, TN_EINVAL, "dims out of range");
            }
        TN_HIP(ctx, hipMemcpyAsync(ctx->env + (size_t)Lx * box, env,
                                   (size_t)(Ly - 1) * Lx * box * sizeof(double),
                                   hipMemcpyHostToDevice, ctx->stream));
        TN_HIP(ctx, hipMemcpyAsync(ctx->dims + (Lx + 1), dims,
                                   (size_t)(Ly - 1) * (Lx + 1) * sizeof(int),
                                   hipMemcpyHostToDevice, ctx->stream));
        if (ell)
            TN_HIP(ctx, hipMemcpyAsync(ctx->ell + 1, ell, (size_t)(Ly - 1) * sizeof(double),
                                       hipMemcpyHostToDevice, ctx->stream));
    }
    std::vector<int> ones(Lx + 1, 1);
    TN_HIP(ctx, hipMemcpyAsync(ctx->dims + (size_t)Ly * (Lx + 1), ones.data(),
                               (Lx + 1) * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if ((rc = tn_make_operands(ctx, prec))) return rc;
    ctx->logZ = logZ;
    ctx->has_env = true;
    return TN_OK;
}

int tn_get_env(tn_ctx *ctx, double *env, int *dims, double *ell, double *logZ) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    const int Lx = ctx->Lx, Ly = ctx->Ly, D = ctx->D;
    const size_t box = (size_t)2 * D * D;
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (Ly > 1) {
        if (env)
            TN_HIP(ctx, hipMemcpy(env, ctx->env + (size_t)Lx * box,
                                  (size_t)(Ly - 1) * Lx * box * sizeof(double),
                                  hipMemcpyDeviceToHost));
        if (dims)
            TN_HIP(ctx, hipMemcpy(dims, ctx->dims + (Lx + 1),
                                  (size_t)(Ly - 1) * (Lx + 1) * sizeof(int), hipMemcpyDeviceToHost));
        if (ell)
            TN_HIP(ctx, hipMemcpy(ell, ctx->ell + 1, (size_t)(Ly - 1) * sizeof(double),
                                  hipMemcpyDeviceToHost));
    }
    if (logZ) *logZ = ctx->logZ;
    return TN_OK;
}

int tn_set_precision(tn_ctx *ctx, int prec) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    if ((rc = check_prec(ctx, prec))) return rc;
    if ((rc = tn_make_operands(ctx, prec))) return rc;
    ctx->prec = prec;
    return TN_OK;
}

int tn_set_instance(tn_ctx *ctx, int inst) {
    if (!ctx) return TN_EINVAL;
    if (inst < 0 || inst >= (1 << 29)) return tn_fail(ctx, TN_EINVAL, "inst out of range");
    ctx->inst = inst;
    return TN_OK;
}

int tn_sample(tn_ctx *ctx, int batch, uint64_t seed, uint64_t step, uint64_t first_id,
              int8_t *spins, double *logq, double *energy) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    ctx->err.clear();
    if (batch < 0) return tn_fail(ctx, TN_EINVAL, "batch < 0");
    if (batch > 0 && (!spins || !logq || !energy))
        return tn_fail(ctx, TN_EINVAL, "NULL output buffer");
    if (ctx->prec == TN_FP64)
        return tn_run_fp64(ctx, batch, seed, step, batch, first_id, spins, false, logq, energy);
    return tn_run_mfma(ctx, batch, seed, step, batch, first_id, spins, false, logq, energy);
}

int tn_eval_logq(tn_ctx *ctx, int batch, const int8_t *spins, double *logq, double *energy) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    ctx->err.clear();
    if (batch < 0) return tn_fail(ctx, TN_EINVAL, "batch < 0");
    if (batch > 0 && (!spins || !logq || !energy))
        return tn_fail(ctx, TN_EINVAL, "NULL buffer");
    int8_t *s = const_cast<int8_t *>(spins);   // read-only in eval mode
    if (ctx->prec == TN_FP64) return tn_run_fp64(ctx, batch, 0, 0, batch, 0, s, true, logq, energy);
    return tn_run_mfma(ctx, batch, 0, 0, batch, 0, s, true, logq, energy);
}

int tn_mh_step(tn_ctx *ctx, int chains, uint64_t seed, uint64_t step, int8_t *state_spins,
               double *state_logq, double *state_energy, uint8_t *accepted) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    ctx->err.clear();
    if (chains < 0) return tn_fail(ctx, TN_EINVAL, "chains < 0");
    if (chains == 0) return TN_OK;
    if (!state_spins || !state_logq || !state_energy || !accepted)
        return tn_fail(ctx, TN_EINVAL, "NULL state buffer");
    const size_t nsite = (size_t)ctx->Lx * ctx->Ly;
    const size_t spin_bytes = ((chains * nsite + 255) / 256) * 256;
    const size_t need = spin_bytes + 2 * (size_t)chains * sizeof(double);
    if (need > ctx->pcap) {
        void *p = ctx->pspins;
        if ((rc = tn_ensure(ctx, &p, &ctx->pcap, need))) return rc;
        ctx->pspins = (int8_t *)p;
    }
    ctx->plogq = (double *)(ctx->pspins + spin_bytes);
    ctx->pE = ctx->plogq + chains;
    if ((rc = tn_sample(ctx, chains, seed, step, 0, ctx->pspins, ctx->plogq, ctx->pE))) return rc;
    return tn_launch_accept(ctx, chains, seed, step, ctx->pspins, ctx->plogq, ctx->pE,
                            state_spins, state_logq, state_energy, accepted);
}

int tn_sample_steps(tn_ctx *ctx, int chains, int nsteps, uint64_t seed, uint64_t step0,
                    uint64_t first_id, int8_t *spins, double *logq, double *energy) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    ctx->err.clear();
    if (chains < 0 || nsteps < 1) return tn_fail(ctx, TN_EINVAL, "chains < 0 or nsteps < 1");
    if ((size_t)chains * nsteps > (size_t)INT32_MAX / 2)
        return tn_fail(ctx, TN_EINVAL, "chains * nsteps too large");
    if (chains == 0) return TN_OK;
    if (!spins || !logq || !energy) return tn_fail(ctx, TN_EINVAL, "NULL output buffer");
    const int batch = chains * nsteps;
    if (ctx->prec == TN_FP64)
        return tn_run_fp64(ctx, batch, seed, step0, chains, first_id, spins, false, logq, energy);
    return tn_run_mfma(ctx, batch, seed, step0, chains, first_id, spins, false, logq, energy);
}

int tn_mh_run(tn_ctx *ctx, int chains, int nsteps, uint64_t seed, uint64_t step0,
              int8_t *state_spins, double *state_logq, double *state_energy,
              uint8_t *accepted, double *energy_series) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    ctx->err.clear();
    if (chains < 0 || nsteps < 0) return tn_fail(ctx, TN_EINVAL, "chains < 0 or nsteps < 0");
    if (chains == 0 || nsteps == 0) return TN_OK;
    if (!state_spins || !state_logq || !state_energy || !accepted)
        return tn_fail(ctx, TN_EINVAL, "NULL state buffer");
    // steps per sampler launch: two 16-proposal workgroups per compute unit
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess)
        cus = 256;
    const long target = 2L * 16 * cus;
    int m = (int)((target + chains - 1) / chains);
    m = m < 1 ? 1 : (m > nsteps ? nsteps : m);
    if ((size_t)chains * m > (size_t)INT32_MAX / 2) m = 1;
    const size_t nsite = (size_t)ctx->Lx * ctx->Ly;
    const size_t spin_bytes = ((m * chains * nsite + 255) / 256) * 256;
    const size_t need = spin_bytes + 2 * (size_t)m * chains * sizeof(double);
    if (need > ctx->pcap) {
        void *p = ctx->pspins;
        if ((rc = tn_ensure(ctx, &p, &ctx->pcap, need))) return rc;
        ctx->pspins = (int8_t *)p;
    }
    ctx->plogq = (double *)(ctx->pspins + spin_bytes);
    ctx->pE = ctx->plogq + (size_t)m * chains;
    for (int t0 = 0; t0 < nsteps; t0 += m) {
        const int mm = nsteps - t0 < m ? nsteps - t0 : m;
        if ((rc = tn_sample_steps(ctx, chains, mm, seed, step0 + t0, 0, ctx->pspins, ctx->plogq,
                                  ctx->pE)))
            return rc;
        for (int j = 0; j < mm; ++j) {
            const size_t o = (size_t)j * chains;
            if ((rc = tn_launch_accept(ctx, chains, seed, step0 + t0 + j, ctx->pspins + o * nsite,
                                       ctx->plogq + o, ctx->pE + o, state_spins, state_logq,
                                       state_energy, accepted + (size_t)(t0 + j) * chains)))
                return rc;
            if (energy_series)
                TN_HIP(ctx, hipMemcpyAsync(energy_series + (size_t)(t0 + j) * chains, state_energy,
                                           (size_t)chains * sizeof(double),
                                           hipMemcpyDeviceToDevice, ctx->stream));
        }
    }
    return TN_OK;
}

int tn_mh_accept(tn_ctx *ctx, int chains, uint64_t seed, uint64_t step,
                 const int8_t *prop_spins, const double *prop_logq, const double *prop_energy,
                 int8_t *state_spins, double *state_logq, double *state_energy,
                 uint8_t *accepted) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    ctx->err.clear();
    if (chains < 0) return tn_fail(ctx, TN_EINVAL, "chains < 0");
    if (chains == 0) return TN_OK;
    if (!prop_spins || !prop_logq || !prop_energy || !state_spins || !state_logq ||
        !state_energy || !accepted)
        return tn_fail(ctx, TN_EINVAL, "NULL buffer");
    return tn_launch_accept(ctx, chains, seed, step, prop_spins, prop_logq, prop_energy,
                            state_spins, state_logq, state_energy, accepted);
}

int tn_grad(tn_ctx *ctx, double *dJh, double *dJv, double *dbeta) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    ctx->err.clear();
    if ((ctx->Lx > 1 && !dJh) || (ctx->Ly > 1 && !dJv))
        return tn_fail(ctx, TN_EINVAL, "NULL gradient buffer");
    return tn_grad_device(ctx, dJh, dJv, dbeta);
}

int tn_stats(tn_ctx *ctx, tn_stats_t *out, int reset) {
    (void)hipGetLastError();
    if (!ctx || !out) return TN_EINVAL;
    unsigned long long c[CNT_N];
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    TN_HIP(ctx, hipMemcpy(c, ctx->counters, sizeof(c), hipMemcpyDeviceToHost));
    out->clamps = c[CNT_CLAMPS];
    out->both_nonpos = c[CNT_BOTH];
    out->near_threshold = c[CNT_NEAR];
    out->accepted = c[CNT_ACCEPTED];
    out->proposed = c[CNT_PROPOSED];
    out->degenerate_cuts = c[CNT_DEGEN];
    out->logZ = ctx->logZ;
    out->env_build_ms = ctx->env_build_ms;
    if (reset) TN_HIP(ctx, hipMemset(ctx->counters, 0, sizeof(c)));
    return TN_OK;
}

}  // extern "C"
