// C ABI entry points (include/tnmh.h): argument checks, ownership of device
// buffers, dispatch to the kernels.  No exception crosses the boundary.
#include "common.hpp"

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

// Scratch of tn_sample_noalloc: a fixed device array of the library (each GPU
// the library runs on holds its own copy until the process ends).  Host code
// never uses the array's name as an address: tn_create takes the address of
// the current device's copy once per device (hipGetSymbolAddress) and every
// later use goes through that pointer.
constexpr size_t TN_NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[TN_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int TN_MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[TN_MAX_DEVICES] = {};
hipError_t g_scratch_err[TN_MAX_DEVICES] = {};
bool g_scratch_done[TN_MAX_DEVICES] = {};

// The address of the current device's scratch copy, looked up on the first
// call for that device; nullptr (and the lookup's error) if it failed.
void *noalloc_scratch(int device, hipError_t *err) {
    if (device < 0 || device >= TN_MAX_DEVICES) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_done[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_err[device] = e;
        g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
        if (e != hipSuccess) (void)hipGetLastError();
        g_scratch_done[device] = true;
    }
    *err = g_scratch_err[device];
    return g_scratch_ptr[device];
}
}  // namespace

int tn_fail(tn_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int tn_ensure(tn_ctx *ctx, void **ptr, size_t *cap, size_t bytes) {
    if (bytes <= *cap && *ptr) return TN_OK;
    if (ctx->capturing)   // no synchronisation or allocation inside a stream capture
        return tn_fail(ctx, TN_ESTATE, "buffers not allocated: run the call once before capture");
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

int tn_multi_prepare(tn_ctx *ctx) {
    int rc;
    for (size_t i = 0; i < ctx->kids.size(); ++i) {
        tn_ctx *k = ctx->kids[i];
        const int C = ctx->kid_chains[i];
        // an instance switched to FP64 operands on the matrix cores
        // (tn_set_precision) has no batched sampler group: refuse it rather
        // than run a group's kernel on its operand layout
        if (k->prec == TN_FP64_MFMA)
            return tn_fail(ctx, TN_EINVAL, "instance " + std::to_string(i) +
                                               " has TN_FP64_MFMA operands: batched steps take TN_FP64, "
                                               "TN_FP32 or TN_BF16");
        const size_t nsite = (size_t)k->Lx * k->Ly;
        const size_t spin_bytes = (((size_t)C * nsite + 255) / 256) * 256;
        const size_t need = spin_bytes + 2 * (size_t)C * sizeof(double);
        const size_t gneed = k->prec == TN_FP64 ? (size_t)C * k->Lx * 2 * k->D * sizeof(double)
                                                : tn_mfma_scratch_bytes(k, C);
        if ((need > k->pcap || gneed > k->gscr_cap) && ctx->capturing)
            return tn_fail(ctx, TN_ESTATE, "buffers not allocated: run the step once before capture");
        if (need > k->pcap) {
            void *p = k->pspins;
            if ((rc = tn_ensure(k, &p, &k->pcap, need))) return tn_fail(ctx, rc, k->err);
            k->pspins = (int8_t *)p;
        }
        if (gneed > k->gscr_cap && (rc = tn_ensure(k, &k->gscr, &k->gscr_cap, gneed)))
            return tn_fail(ctx, rc, k->err);
        k->plogq = (double *)(k->pspins + spin_bytes);
        k->pE = k->plogq + C;
    }
    return TN_OK;
}

void tn_multi_groups(tn_ctx *ctx, std::vector<tn_samp_desc> &sd, std::vector<tn_multi_group> &groups) {
    for (int bf = 0; bf < 2; ++bf)
        for (int NT = 1; NT <= 4; ++NT) {
            tn_multi_group g{NT, bf == 1, (int)sd.size(), 0, 0, 1};
            for (size_t i = 0; i < ctx->kids.size(); ++i) {
                tn_ctx *k = ctx->kids[i];
                const int C = ctx->kid_chains[i];
                if (k->prec == TN_FP64 || C == 0 || k->Dp / 16 != NT || (k->prec == TN_BF16) != (bf == 1))
                    continue;
                tn_samp_desc A = tn_samp_desc_of(k, C, k->pspins, k->plogq, k->pE,
                                                 (float *)k->gscr, C, 0);
                A.blk0 = g.blocks;   // in 16-proposal units, whole teams (up to eight units) per instance
                g.blocks += ((C + 127) / 128) * 8;
                g.maxLx = k->Lx > g.maxLx ? k->Lx : g.maxLx;
                sd.push_back(A);
                ++g.count;
            }
            if (g.count) groups.push_back(g);
        }
}

namespace {

void free_all(tn_ctx *ctx) {
    tn_periodic_free(ctx);
    for (tn_ctx *k : ctx->kids) {
        free_all(k);
        delete k;
    }
    if (ctx->flip) {
        free_all(ctx->flip);
        delete ctx->flip;
        ctx->flip = nullptr;
    }
    ctx->kids.clear();
    for (tn_ctx *k : ctx->fkids) {
        free_all(k);
        delete k;
    }
    ctx->fkids.clear();
    void *bufs[] = {ctx->Jh,    ctx->Jv,   ctx->h,    ctx->env,  ctx->dims,   ctx->ell,
                    ctx->G64r,  ctx->G32R, ctx->G16R, ctx->G64MR, ctx->fac,  ctx->xbox,   ctx->wbuf,
                    ctx->scal,  ctx->xdims, ctx->gscr, ctx->pspins, ctx->counters,
                    ctx->cst,   ctx->gradscr, ctx->descs, ctx->fbuf, ctx->pscr,
                    ctx->pq,    ctx->pG,   ctx->pw,
                    ctx->own_dstep ? (void *)ctx->dstep : nullptr};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
    for (void *p : ctx->mdesc) (void)hipFree(p);
    ctx->mdesc.clear();
    ctx->mdesc_host.clear();
    delete (tn_build_plan *)ctx->build_plan;
    ctx->build_plan = nullptr;
}

}  // namespace

void tn_free_ctx(tn_ctx *ctx) { free_all(ctx); }

namespace {

int check_prec(tn_ctx *ctx, int prec) {
    if (prec != TN_FP64 && prec != TN_FP32 && prec != TN_BF16 && prec != TN_FP64_MFMA)
        return tn_fail(ctx, TN_EINVAL, "prec must be TN_FP64, TN_FP32, TN_BF16 or TN_FP64_MFMA");
    return TN_OK;
}

// Copy the couplings into context-owned buffers and record the instance.
int set_instance(tn_ctx *ctx, int Lx, int Ly, const double *Jh, const double *Jv,
                 const double *h, double beta, int D, int prec) {
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "not allowed while capturing a graph");
    ctx->qd = 0;             // an Ising instance
    ctx->building = false;   // a new instance abandons an open incremental build
    ++ctx->env_gen;
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

// tn_sample after the common checks; tn_mh_step calls it while capturing
int sample_impl(tn_ctx *ctx, int batch, uint64_t seed, uint64_t step, uint64_t first_id,
                int8_t *spins, double *logq, double *energy) {
    if (batch < 0) return tn_fail(ctx, TN_EINVAL, "batch < 0");
    if (batch > 0 && (!spins || !logq || !energy))
        return tn_fail(ctx, TN_EINVAL, "NULL output buffer");
    if (ctx->qd) return tn_run_potts(ctx, batch, seed, step, batch, first_id, spins, false, logq, energy);
    if (ctx->prec == TN_FP64)
        return tn_run_fp64(ctx, batch, seed, step, batch, first_id, spins, false, logq, energy);
    return tn_run_mfma(ctx, batch, seed, step, batch, first_id, spins, false, logq, energy);
}

// calls defined for Ising contexts only
int not_potts(tn_ctx *ctx) {
    if (ctx->qd) return tn_fail(ctx, TN_EINVAL, "not available for a Potts context (tn_potts_build_env)");
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
        hipMalloc((void **)&ctx->dstep, sizeof(uint64_t)) != hipSuccess ||
        hipMemset(ctx->dstep, 0, sizeof(uint64_t)) != hipSuccess ||
        hipMalloc((void **)&ctx->xdims, 4096 * sizeof(int)) != hipSuccess ||
        hipMemset(ctx->counters, 0, CNT_N * sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        free_all(ctx);
        delete ctx;
        return TN_EHIP;
    }
    // the no-allocation sampler's scratch on this device (looked up once per
    // device, with the device current); a failed lookup only disables
    // tn_sample_noalloc, which reports it
    hipError_t se = hipSuccess;
    ctx->noalloc_scr = noalloc_scratch(ctx->device, &se);
    ctx->noalloc_err = (int)se;
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
    ctx->has_cst = ctx->fit_sweeps == 0;   // the frozen derivative needs SVD cuts
    if (logZ_out) {
        TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
        *logZ_out = lz;
    }
    return TN_OK;
}

int tn_build_env_begin(tn_ctx *ctx, int Lx, int Ly, const double *Jh, const double *Jv,
                       const double *h, double beta, int D, int prec) {
    (void)hipGetLastError();
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "not allowed while capturing a graph");
    int rc;
    ctx->building = false;
    if ((rc = set_instance(ctx, Lx, Ly, Jh, Jv, h, beta, D, prec))) return rc;
    if (!ctx->build_plan) ctx->build_plan = new (std::nothrow) tn_build_plan();
    if (!ctx->build_plan) return tn_fail(ctx, TN_ENOMEM, "out of host memory");
    tn_ctx *one[1] = {ctx};
    std::string e;
    if ((rc = tn_env_build_prepare(one, 1, ctx->stream, &e, (tn_build_plan *)ctx->build_plan)))
        return tn_fail(ctx, rc, e);
    ctx->build_step = 0;
    ctx->building = true;
    return TN_OK;
}

int tn_build_env_rows(tn_ctx *ctx, int nrows, int *rows_left) {
    (void)hipGetLastError();
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    if (!ctx->building) return tn_fail(ctx, TN_ESTATE, "no build open: call tn_build_env_begin");
    if (nrows < 0) return tn_fail(ctx, TN_EINVAL, "nrows < 0");
    tn_build_plan *plan = (tn_build_plan *)ctx->build_plan;
    const int total = plan->maxLy - 1;
    const int s1 = ctx->build_step + nrows < total ? ctx->build_step + nrows : total;
    std::string e;
    int rc;
    if ((rc = tn_env_build_steps(plan, ctx->build_step, s1, ctx->stream, &e))) {
        ctx->building = false;
        return tn_fail(ctx, rc, e);
    }
    ctx->build_step = s1;
    if (rows_left) *rows_left = total - s1;
    return TN_OK;
}

int tn_build_env_end(tn_ctx *ctx, double *logZ_out) {
    (void)hipGetLastError();
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    if (!ctx->building) return tn_fail(ctx, TN_ESTATE, "no build open: call tn_build_env_begin");
    int rc, left = 0;
    if ((rc = tn_build_env_rows(ctx, 1 << 30, &left))) return rc;
    ctx->building = false;
    tn_ctx *one[1] = {ctx};
    std::string e;
    if ((rc = tn_env_build_finish(one, 1, (tn_build_plan *)ctx->build_plan, ctx->stream, &e)))
        return tn_fail(ctx, rc, e);
    if ((rc = tn_make_operands(ctx, ctx->prec))) return rc;
    ctx->has_env = true;
    ctx->has_cst = ctx->fit_sweeps == 0;   // the frozen derivative needs SVD cuts
    if (logZ_out) *logZ_out = ctx->logZ;
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
    if ((rc = not_potts(ctx))) return rc;
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "not allowed while capturing a graph");
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
    if ((rc = not_potts(ctx))) return rc;
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "not allowed while capturing a graph");
    if ((rc = check_prec(ctx, prec))) return rc;
    if ((rc = tn_make_operands(ctx, prec))) return rc;
    ctx->prec = prec;
    return TN_OK;
}

int tn_set_compression(tn_ctx *ctx, int fit_sweeps) {
    (void)hipGetLastError();
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    if (fit_sweeps < 0 || fit_sweeps > 16) return tn_fail(ctx, TN_EINVAL, "fit_sweeps must be in 0..16");
    ctx->fit_sweeps = fit_sweeps;
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
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "only MH steps may be captured");
    return sample_impl(ctx, batch, seed, step, first_id, spins, logq, energy);
}

int tn_sample_noalloc(tn_ctx *ctx, int batch, uint64_t seed, uint64_t step, uint64_t first_id,
                      int8_t *spins, double *logq, double *energy) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    ctx->err.clear();
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "only MH steps may be captured");
    if (batch < 0) return tn_fail(ctx, TN_EINVAL, "batch < 0");
    if (batch == 0) return TN_OK;
    if (!spins || !logq || !energy) return tn_fail(ctx, TN_EINVAL, "NULL output buffer");
    if (!ctx->noalloc_scr)
        return tn_fail(ctx, TN_EHIP, std::string("address of the fixed scratch not available: ") +
                                         hipGetErrorString((hipError_t)ctx->noalloc_err));
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != ctx->device)
        return tn_fail(ctx, TN_EINVAL, "the context's device must be current");
    const size_t need = ctx->qd ? tn_potts_scratch_bytes(ctx, batch)
                                : (ctx->prec == TN_FP64 ? tn_fp64_scratch_bytes(ctx, batch)
                                                        : tn_mfma_scratch_bytes(ctx, batch));
    if (need > TN_NOALLOC_SCRATCH_BYTES)
        return tn_fail(ctx, TN_EINVAL, "tn_sample_noalloc: " + std::to_string(batch) +
                                           " proposals need " + std::to_string(need) +
                                           " bytes of scratch, above its fixed " +
                                           std::to_string(TN_NOALLOC_SCRATCH_BYTES) + " bytes");
    if (ctx->qd)
        return tn_run_potts(ctx, batch, seed, step, batch, first_id, spins, false, logq, energy,
                            ctx->noalloc_scr);
    if (ctx->prec == TN_FP64)
        return tn_run_fp64(ctx, batch, seed, step, batch, first_id, spins, false, logq, energy,
                           ctx->noalloc_scr);
    return tn_run_mfma(ctx, batch, seed, step, batch, first_id, spins, false, logq, energy, -1,
                       ctx->noalloc_scr);
}

int tn_eval_logq(tn_ctx *ctx, int batch, const int8_t *spins, double *logq, double *energy) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    ctx->err.clear();
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "only MH steps may be captured");
    if (batch < 0) return tn_fail(ctx, TN_EINVAL, "batch < 0");
    if (batch > 0 && (!spins || !logq || !energy))
        return tn_fail(ctx, TN_EINVAL, "NULL buffer");
    int8_t *s = const_cast<int8_t *>(spins);   // read-only in eval mode
    if (ctx->qd) return tn_run_potts(ctx, batch, 0, 0, batch, 0, s, true, logq, energy);
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
        if (ctx->capturing)
            return tn_fail(ctx, TN_ESTATE, "buffers not allocated: run the step once before capture");
        void *p = ctx->pspins;
        if ((rc = tn_ensure(ctx, &p, &ctx->pcap, need))) return rc;
        ctx->pspins = (int8_t *)p;
    }
    ctx->plogq = (double *)(ctx->pspins + spin_bytes);
    ctx->pE = ctx->plogq + chains;
    if ((rc = sample_impl(ctx, chains, seed, step, 0, ctx->pspins, ctx->plogq, ctx->pE))) return rc;
    if ((rc = tn_launch_accept(ctx, chains, seed, step, ctx->pspins, ctx->plogq, ctx->pE,
                               state_spins, state_logq, state_energy, accepted)))
        return rc;
    if (ctx->capturing) ++ctx->graph_steps;
    return TN_OK;
}

int tn_sample_steps(tn_ctx *ctx, int chains, int nsteps, uint64_t seed, uint64_t step0,
                    uint64_t first_id, int8_t *spins, double *logq, double *energy) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    ctx->err.clear();
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "only MH steps may be captured");
    if (chains < 0 || nsteps < 1) return tn_fail(ctx, TN_EINVAL, "chains < 0 or nsteps < 1");
    if ((size_t)chains * nsteps > (size_t)INT32_MAX / 2)
        return tn_fail(ctx, TN_EINVAL, "chains * nsteps too large");
    if (chains == 0) return TN_OK;
    if (!spins || !logq || !energy) return tn_fail(ctx, TN_EINVAL, "NULL output buffer");
    const int batch = chains * nsteps;
    if (ctx->qd) return tn_run_potts(ctx, batch, seed, step0, chains, first_id, spins, false, logq, energy);
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
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "only MH steps may be captured");
    if (chains < 0 || nsteps < 0) return tn_fail(ctx, TN_EINVAL, "chains < 0 or nsteps < 0");
    if (chains == 0 || nsteps == 0) return TN_OK;
    if (!state_spins || !state_logq || !state_energy || !accepted)
        return tn_fail(ctx, TN_EINVAL, "NULL state buffer");
    // steps per sampler launch: the autotuned proposals per launch, else two
    // teams of 128 proposals for every compute unit
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess)
        cus = 256;
    const long target = tn_tuned_here(ctx) ? ctx->tuned.proposals : 16L * 16 * cus;
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
                                       state_energy, accepted + (size_t)(t0 + j) * chains,
                                       energy_series ? energy_series + (size_t)(t0 + j) * chains
                                                     : nullptr)))
                return rc;
        }
    }
    return TN_OK;
}

int tn_metropolis_sweeps(tn_ctx *ctx, int chains, int nsweeps, uint64_t seed, uint64_t step,
                         int8_t *state_spins, double *state_logq, double *state_energy) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    if ((rc = not_potts(ctx))) return rc;
    ctx->err.clear();
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "only MH steps may be captured");
    if (chains < 0 || nsweeps < 0) return tn_fail(ctx, TN_EINVAL, "chains < 0 or nsweeps < 0");
    if (nsweeps >= (1 << 18)) return tn_fail(ctx, TN_EINVAL, "nsweeps must be below 2^18");
    if ((long)ctx->Lx * ctx->Ly > 65536) return tn_fail(ctx, TN_EINVAL, "more than 65536 sites");
    if (chains == 0 || nsweeps == 0) return TN_OK;
    if (!state_spins || !state_logq || !state_energy) return tn_fail(ctx, TN_EINVAL, "NULL state buffer");
    if ((rc = tn_launch_metropolis(ctx, chains, nsweeps, seed, step, state_spins))) return rc;
    // ln q and E of the new states, by the arithmetic that draws the proposals
    if (ctx->prec == TN_FP64)
        return tn_run_fp64(ctx, chains, 0, 0, chains, 0, state_spins, true, state_logq, state_energy);
    return tn_run_mfma(ctx, chains, 0, 0, chains, 0, state_spins, true, state_logq, state_energy);
}

int tn_link_overlap(tn_ctx *ctx, int n, const int8_t *a, const int8_t *b, int32_t *q) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    if ((rc = not_potts(ctx))) return rc;
    ctx->err.clear();
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "only MH steps may be captured");
    if (n < 0) return tn_fail(ctx, TN_EINVAL, "n < 0");
    if (n == 0) return TN_OK;
    if (!a || !b || !q) return tn_fail(ctx, TN_EINVAL, "NULL buffer");
    return tn_launch_link_overlap(ctx, n, a, b, q);
}

int tn_mh_accept(tn_ctx *ctx, int chains, uint64_t seed, uint64_t step,
                 const int8_t *prop_spins, const double *prop_logq, const double *prop_energy,
                 int8_t *state_spins, double *state_logq, double *state_energy,
                 uint8_t *accepted) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    ctx->err.clear();
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "only MH steps may be captured");
    if (chains < 0) return tn_fail(ctx, TN_EINVAL, "chains < 0");
    if (chains == 0) return TN_OK;
    if (!prop_spins || !prop_logq || !prop_energy || !state_spins || !state_logq ||
        !state_energy || !accepted)
        return tn_fail(ctx, TN_EINVAL, "NULL buffer");
    return tn_launch_accept(ctx, chains, seed, step, prop_spins, prop_logq, prop_energy,
                            state_spins, state_logq, state_energy, accepted);
}

// ---- batched uneven instances -------------------------------------------

int tn_build_env_multi(tn_ctx *ctx, int n, const tn_instance *inst, int prec, double *logZ_out) {
    (void)hipGetLastError();
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "not allowed while capturing a graph");
    if (n < 1 || !inst) return tn_fail(ctx, TN_EINVAL, "need n >= 1 instances");
    int rc;
    if ((rc = check_prec(ctx, prec))) return rc;
    if (prec == TN_FP64_MFMA)
        return tn_fail(ctx, TN_EINVAL, "batched instances take TN_FP64, TN_FP32 or TN_BF16");
    for (int i = 0; i < n; ++i)
        if (inst[i].chains < 0) return tn_fail(ctx, TN_EINVAL, "chains < 0");
    while ((int)ctx->kids.size() > n) {
        tn_ctx *k = ctx->kids.back();
        ctx->kids.pop_back();
        free_all(k);
        delete k;
    }
    while ((int)ctx->kids.size() < n) {
        tn_ctx *k = new (std::nothrow) tn_ctx();
        if (!k) return tn_fail(ctx, TN_ENOMEM, "out of host memory");
        k->stream = ctx->stream;
        k->device = ctx->device;
        k->dstep = ctx->dstep;   // the instances follow the batched context's step base
        k->own_dstep = false;
        k->noalloc_scr = ctx->noalloc_scr;   // same device, same fixed scratch
        k->noalloc_err = ctx->noalloc_err;
        ctx->kids.push_back(k);
        if (hipMalloc((void **)&k->counters, CNT_N * sizeof(unsigned long long)) != hipSuccess ||
            hipMalloc((void **)&k->scal, 16 * sizeof(double)) != hipSuccess ||
            hipMalloc((void **)&k->xdims, 4096 * sizeof(int)) != hipSuccess ||
            hipMemset(k->counters, 0, CNT_N * sizeof(unsigned long long)) != hipSuccess) {
            (void)hipGetLastError();
            return tn_fail(ctx, TN_ENOMEM, "device allocation failed");
        }
    }
    ctx->has_multi = false;
    ctx->kid_chains.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        tn_ctx *k = ctx->kids[i];
        k->err.clear();
        k->has_env = false;
        const tn_instance &I = inst[i];
        if ((rc = set_instance(k, I.Lx, I.Ly, I.Jh, I.Jv, I.h, I.beta, I.D, prec)))
            return tn_fail(ctx, rc, "instance " + std::to_string(i) + ": " + k->err);
        k->inst = i;
        k->fit_sweeps = ctx->fit_sweeps;
        ctx->kid_chains[i] = I.chains;
    }
    std::string e;
    if ((rc = tn_env_build_many(ctx->kids.data(), n, ctx->stream, &e))) return tn_fail(ctx, rc, e);
    for (int i = 0; i < n; ++i) {
        tn_ctx *k = ctx->kids[i];
        if ((rc = tn_make_operands(k, prec)))
            return tn_fail(ctx, rc, "instance " + std::to_string(i) + ": " + k->err);
        k->has_env = true;
        k->has_cst = k->fit_sweeps == 0;
        if (logZ_out) logZ_out[i] = k->logZ;
    }
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (void *p : ctx->mdesc) (void)hipFree(p);
    ctx->mdesc.clear();
    ctx->mdesc_host.clear();
    ctx->has_multi = true;
    return TN_OK;
}

int tn_mh_step_multi(tn_ctx *ctx, uint64_t seed, uint64_t step, int8_t *const *state_spins,
                     double *const *state_logq, double *const *state_energy,
                     uint8_t *const *accepted) {
    (void)hipGetLastError();
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    if (!ctx->has_multi) return tn_fail(ctx, TN_ESTATE, "no instances: call tn_build_env_multi first");
    if (!state_spins || !state_logq || !state_energy || !accepted)
        return tn_fail(ctx, TN_EINVAL, "NULL state array");
    const int n = (int)ctx->kids.size();
    int rc;
    for (int i = 0; i < n; ++i)
        if (ctx->kid_chains[i] > 0 && (!state_spins[i] || !state_logq[i] || !state_energy[i] || !accepted[i]))
            return tn_fail(ctx, TN_EINVAL, "NULL state buffer of instance " + std::to_string(i));
    if ((rc = tn_multi_prepare(ctx))) return rc;
    std::vector<tn_samp_desc> sd;
    std::vector<tn_multi_group> groups;
    tn_multi_groups(ctx, sd, groups);
    std::vector<tn_acc_desc> ad;
    int total = 0;
    for (int i = 0; i < n; ++i) {
        tn_ctx *k = ctx->kids[i];
        const int C = ctx->kid_chains[i];
        if (C == 0) continue;
        tn_acc_desc A;
        A.chains = C;
        A.nsite = k->Lx * k->Ly;
        A.beta = k->beta;
        A.inst = (uint32_t)k->inst;
        A.blk0 = total;
        A.pspins = k->pspins;
        A.plogq = k->plogq;
        A.pE = k->pE;
        A.sspins = state_spins[i];
        A.slogq = state_logq[i];
        A.sE = state_energy[i];
        A.accepted = accepted[i];
        A.counters = k->counters;
        A.eser = nullptr;
        ad.push_back(A);
        total += C;
    }
    const size_t sbytes = sd.size() * sizeof(tn_samp_desc);
    const size_t abytes = ad.size() * sizeof(tn_acc_desc);
    std::vector<unsigned char> host(sbytes + abytes);
    if (sbytes) memcpy(host.data(), sd.data(), sbytes);
    if (abytes) memcpy(host.data() + sbytes, ad.data(), abytes);
    int slot = -1;
    for (size_t q = 0; q < ctx->mdesc_host.size(); ++q)
        if (ctx->mdesc_host[q] == host) slot = (int)q;
    if (slot < 0) {
        if (ctx->capturing)
            return tn_fail(ctx, TN_ESTATE,
                           "state buffers not seen before capture: run the step once first");
        if ((int)ctx->mdesc.size() >= TN_MDESC_SETS) {   // forget the oldest set
            (void)hipFree(ctx->mdesc.front());
            ctx->mdesc.erase(ctx->mdesc.begin());
            ctx->mdesc_host.erase(ctx->mdesc_host.begin());
        }
        void *p = nullptr;
        TN_HIP(ctx, hipMalloc(&p, host.size() ? host.size() : 16));
        ctx->mdesc.push_back(p);
        ctx->mdesc_host.push_back(host);
        if (host.size())
            TN_HIP(ctx, hipMemcpy(p, host.data(), host.size(), hipMemcpyHostToDevice));
        slot = (int)ctx->mdesc.size() - 1;
    }
    const tn_samp_desc *sdev = (const tn_samp_desc *)ctx->mdesc[slot];
    const tn_acc_desc *adev = (const tn_acc_desc *)((unsigned char *)ctx->mdesc[slot] + sbytes);
    for (const tn_multi_group &g : groups) {
        const int v = ctx->multi_variant[g.bf16 ? 1 : 0][g.NT];
        if ((rc = tn_run_mfma_multi(ctx, g.NT, g.bf16, v < 0 ? 0 : v, sdev + g.first, g.count, g.blocks,
                                    g.maxLx, seed, step)))
            return rc;
    }
    for (int i = 0; i < n; ++i) {   // plain fp64 instances: one sampler launch each
        tn_ctx *k = ctx->kids[i];
        const int C = ctx->kid_chains[i];
        if (k->prec != TN_FP64 || C == 0) continue;
        if ((rc = tn_run_fp64(k, C, seed, step, C, 0, k->pspins, false, k->plogq, k->pE)))
            return tn_fail(ctx, rc, k->err);
    }
    if ((rc = tn_launch_accept_multi(ctx, adev, (int)ad.size(), total, seed, step))) return rc;
    if (ctx->capturing) ++ctx->graph_steps;
    return TN_OK;
}

tn_ctx *tn_multi_instance(tn_ctx *ctx, int i) {
    if (!ctx || i < 0 || i >= (int)ctx->kids.size() || !ctx->has_multi) return nullptr;
    return ctx->kids[i];
}

namespace {
__global__ void k_advance_step(unsigned long long *base, unsigned long long by) {
    if (threadIdx.x == 0) atomicAdd(base, by);
}
}  // namespace

int tn_graph_begin(tn_ctx *ctx) {
    (void)hipGetLastError();
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "a capture is already open");
    if (!ctx->stream)
        return tn_fail(ctx, TN_EINVAL, "graph capture needs a context stream other than the default");
    TN_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    ctx->capturing = true;
    ctx->graph_steps = 0;
    return TN_OK;
}

int tn_graph_end_and_replay(tn_ctx *ctx, int n_replays) {
    (void)hipGetLastError();
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    if (!ctx->capturing) return tn_fail(ctx, TN_ESTATE, "no capture is open");
    // the last node moves the step base on by the captured step count
    hipLaunchKernelGGL(k_advance_step, dim3(1), dim3(64), 0, ctx->stream,
                       (unsigned long long *)ctx->dstep, (unsigned long long)ctx->graph_steps);
    const hipError_t le = hipGetLastError();
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(ctx->stream, &graph);
    ctx->capturing = false;
    if (le != hipSuccess || ee != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return tn_fail(ctx, TN_EHIP, "graph capture failed");
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return tn_fail(ctx, TN_EHIP, "graph instantiation failed");
    }
    int rc = TN_OK;
    if (n_replays < 0) rc = tn_fail(ctx, TN_EINVAL, "n_replays < 0");
    // replays start from the captured steps; afterwards the base is 0 again
    if (rc == TN_OK && hipMemsetAsync(ctx->dstep, 0, sizeof(uint64_t), ctx->stream) != hipSuccess)
        rc = tn_fail(ctx, TN_EHIP, "step base reset failed");
    for (int r = 0; rc == TN_OK && r < n_replays; ++r)
        if (hipGraphLaunch(exec, ctx->stream) != hipSuccess) rc = tn_fail(ctx, TN_EHIP, "graph launch failed");
    if (hipMemsetAsync(ctx->dstep, 0, sizeof(uint64_t), ctx->stream) != hipSuccess && rc == TN_OK)
        rc = tn_fail(ctx, TN_EHIP, "step base reset failed");
    if (hipStreamSynchronize(ctx->stream) != hipSuccess && rc == TN_OK)
        rc = tn_fail(ctx, TN_EHIP, "graph replay failed");
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return rc;
}

int tn_grad(tn_ctx *ctx, double *dJh, double *dJv, double *dbeta) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    if ((rc = not_potts(ctx))) return rc;
    ctx->err.clear();
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "not allowed while capturing a graph");
    if ((ctx->Lx > 1 && !dJh) || (ctx->Ly > 1 && !dJv))
        return tn_fail(ctx, TN_EINVAL, "NULL gradient buffer");
    return tn_grad_device(ctx, nullptr, dJh, dJv, dbeta);
}

int tn_grad_two_sided(tn_ctx *ctx, double *dJh, double *dJv, double *dbeta) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    if ((rc = not_potts(ctx))) return rc;
    ctx->err.clear();
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "not allowed while capturing a graph");
    if ((ctx->Lx > 1 && !dJh) || (ctx->Ly > 1 && !dJv))
        return tn_fail(ctx, TN_EINVAL, "NULL gradient buffer");
    const int Lx = ctx->Lx, Ly = ctx->Ly;
    if (ctx->flip_gen != ctx->env_gen) {
        if (!ctx->flip) {
            ctx->flip = new (std::nothrow) tn_ctx();
            if (!ctx->flip) return tn_fail(ctx, TN_ENOMEM, "out of host memory");
            tn_ctx *f = ctx->flip;
            f->stream = ctx->stream;
            f->device = ctx->device;
            if (hipMalloc((void **)&f->counters, CNT_N * sizeof(unsigned long long)) != hipSuccess ||
                hipMalloc((void **)&f->scal, 16 * sizeof(double)) != hipSuccess ||
                hipMalloc((void **)&f->dstep, sizeof(uint64_t)) != hipSuccess ||
                hipMalloc((void **)&f->xdims, 4096 * sizeof(int)) != hipSuccess ||
                hipMemset(f->counters, 0, CNT_N * sizeof(unsigned long long)) != hipSuccess) {
                (void)hipGetLastError();
                free_all(f);
                delete f;
                ctx->flip = nullptr;
                return tn_fail(ctx, TN_ENOMEM, "allocation for the upside-down build failed");
            }
        }
        // the same couplings with the rows in reverse order
        const size_t nh = (size_t)Ly * (Lx - 1), nv = (size_t)(Ly - 1) * Lx;
        std::vector<double> hJh(nh), hJv(nv), fJh(nh), fJv(nv), hh, fh;
        TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (nh) TN_HIP(ctx, hipMemcpy(hJh.data(), ctx->Jh, nh * sizeof(double), hipMemcpyDeviceToHost));
        if (nv) TN_HIP(ctx, hipMemcpy(hJv.data(), ctx->Jv, nv * sizeof(double), hipMemcpyDeviceToHost));
        for (int r = 0; r < Ly; ++r)
            for (int c = 0; c + 1 < Lx; ++c) fJh[(size_t)r * (Lx - 1) + c] = hJh[(size_t)(Ly - 1 - r) * (Lx - 1) + c];
        for (int r = 0; r + 1 < Ly; ++r)
            for (int c = 0; c < Lx; ++c) fJv[(size_t)r * Lx + c] = hJv[(size_t)(Ly - 2 - r) * Lx + c];
        if (ctx->h) {
            hh.resize((size_t)Ly * Lx);
            fh.resize(hh.size());
            TN_HIP(ctx, hipMemcpy(hh.data(), ctx->h, hh.size() * sizeof(double), hipMemcpyDeviceToHost));
            for (int r = 0; r < Ly; ++r)
                for (int c = 0; c < Lx; ++c) fh[(size_t)r * Lx + c] = hh[(size_t)(Ly - 1 - r) * Lx + c];
        }
        tn_ctx *f = ctx->flip;
        f->err.clear();
        f->fit_sweeps = ctx->fit_sweeps;   // the same compression top-down
        rc = set_instance(f, Lx, Ly, nh ? fJh.data() : nullptr, nv ? fJv.data() : nullptr,
                          ctx->h ? fh.data() : nullptr, ctx->beta, ctx->D, TN_FP64);
        if (rc == TN_OK) rc = tn_env_build_device(f, nullptr);
        // set_instance copied from these host vectors on the stream
        if (hipStreamSynchronize(ctx->stream) != hipSuccess && rc == TN_OK) rc = TN_EHIP;
        if (rc != TN_OK) return tn_fail(ctx, rc, "upside-down build: " + f->err);
        ctx->flip_gen = ctx->env_gen;
    }
    return tn_grad_device(ctx, ctx->flip, dJh, dJv, dbeta);
}

int tn_logz_frozen(tn_ctx *ctx, int n, const double *const *Jh, const double *const *Jv,
                   const double *const *h, const double *beta, double *logZ_out) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_env(ctx))) return rc;
    if ((rc = not_potts(ctx))) return rc;
    ctx->err.clear();
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "not allowed while capturing a graph");
    if (!ctx->has_cst)
        return tn_fail(ctx, TN_ESTATE, "the frozen contraction needs an environment built by tn_build_env "
                                       "with successive SVD");
    if (n < 1 || !beta || !logZ_out) return tn_fail(ctx, TN_EINVAL, "need n >= 1, beta and logZ_out");
    const int Lx = ctx->Lx, Ly = ctx->Ly;
    if ((Lx > 1 && !Jh) || (Ly > 1 && !Jv)) return tn_fail(ctx, TN_EINVAL, "Jh or Jv is NULL");
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(beta[i])) return tn_fail(ctx, TN_EINVAL, "beta must be finite");
        if ((Lx > 1 && !Jh[i]) || (Ly > 1 && !Jv[i]))
            return tn_fail(ctx, TN_EINVAL, "coupling set " + std::to_string(i) + " has a NULL array");
    }
    // one context per evaluation (kept for later calls), built together with
    // the projectors of this context's build
    while ((int)ctx->fkids.size() < n) {
        tn_ctx *k = new (std::nothrow) tn_ctx();
        if (!k) return tn_fail(ctx, TN_ENOMEM, "out of host memory");
        k->stream = ctx->stream;
        k->device = ctx->device;
        ctx->fkids.push_back(k);
        if (hipMalloc((void **)&k->counters, CNT_N * sizeof(unsigned long long)) != hipSuccess ||
            hipMalloc((void **)&k->scal, 16 * sizeof(double)) != hipSuccess ||
            hipMalloc((void **)&k->dstep, sizeof(uint64_t)) != hipSuccess ||
            hipMalloc((void **)&k->xdims, 4096 * sizeof(int)) != hipSuccess ||
            hipMemsetAsync(k->counters, 0, CNT_N * sizeof(unsigned long long), ctx->stream) != hipSuccess) {
            (void)hipGetLastError();
            return tn_fail(ctx, TN_ENOMEM, "allocation for the frozen evaluations failed");
        }
    }
    std::vector<tn_ctx *> ks(ctx->fkids.begin(), ctx->fkids.begin() + n);
    for (int i = 0; i < n; ++i) {
        tn_ctx *k = ks[i];
        k->err.clear();
        k->fit_sweeps = 0;
        k->proj_src = ctx;
        if ((rc = set_instance(k, Lx, Ly, Lx > 1 ? Jh[i] : nullptr, Ly > 1 ? Jv[i] : nullptr,
                               h ? h[i] : nullptr, beta[i], ctx->D, TN_FP64)))
            return tn_fail(ctx, rc, "coupling set " + std::to_string(i) + ": " + k->err);
    }
    std::string e;
    if ((rc = tn_env_build_many(ks.data(), n, ctx->stream, &e))) return tn_fail(ctx, rc, e);
    for (int i = 0; i < n; ++i) logZ_out[i] = ks[i]->logZ;
    return TN_OK;
}

int tn_stats(tn_ctx *ctx, tn_stats_t *out, int reset) {
    (void)hipGetLastError();
    if (!ctx || !out) return TN_EINVAL;
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "not allowed while capturing a graph");
    unsigned long long c[CNT_N];
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    TN_HIP(ctx, hipMemcpy(c, ctx->counters, sizeof(c), hipMemcpyDeviceToHost));
    out->clamps = c[CNT_CLAMPS];
    out->both_nonpos = c[CNT_BOTH];
    out->near_threshold = c[CNT_NEAR];
    out->accepted = c[CNT_ACCEPTED];
    out->proposed = c[CNT_PROPOSED];
    out->degenerate_cuts = c[CNT_DEGEN];
    out->metropolis_flips = c[CNT_FLIPS];
    out->logZ = ctx->logZ;
    out->env_build_ms = ctx->env_build_ms;
    if (reset) TN_HIP(ctx, hipMemset(ctx->counters, 0, sizeof(c)));
    return TN_OK;
}

}  // extern "C"
