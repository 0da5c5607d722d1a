// Autotuner of the batched sampler's launch shape (host code).
//
// The team kernel comes in launch variants that share the arithmetic of a
// proposal and differ in how proposals are packed onto the chip (sets of 16
// proposals per wavefront, wavefronts per SIMD; sampler_mfma.hip).  Which one
// is fastest depends on the lattice, D, the precision and how many proposals
// one launch draws, so it is measured: every candidate is launched on the
// context's own instance and timed with HIP events.  For tn_mh_run the count
// of MH steps whose proposals share a launch is tuned along with it
// (proposals do not depend on the chains' state, Sec. 2, so drawing several
// steps ahead leaves the chains unchanged): the pair that runs the caller's
// max_steps steps fastest wins, launches of m steps plus one of the remainder
// (a launch that fills only part of the chip's team slots costs nearly as
// much as a full one).  tn_autotune_multi tunes the variant of each group's
// one-step launch by its time.
//
// Choices persist in a JSON file: one object whose members are keyed by the
// device architecture and the problem, one member per line,
//   "gfx950|64x64|D32|fp32|chains4096|steps16": {"variant": 0, "proposals": 65536, "ns_per_proposal": 466.1}
// A key found there is used without timing; a new choice is added and the
// file rewritten (through a temporary file renamed over it).
#include "common.hpp"

#include <unistd.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <vector>

namespace {

struct Choice {
    int variant = 0;
    long proposals = 0;
    double ns = 0.0;   // per proposal
};

std::string arch_name(int device) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

const char *prec_name(int prec) {
    return prec == TN_FP64 ? "fp64" : prec == TN_FP32 ? "fp32" : prec == TN_BF16 ? "bf16" : "fp64mfma";
}

std::map<std::string, Choice> read_cache(const char *path) {
    std::map<std::string, Choice> m;
    FILE *f = fopen(path, "r");
    if (!f) return m;
    char line[8192];
    while (fgets(line, sizeof line, f)) {
        const char *q0 = strchr(line, '"');
        if (!q0) continue;
        const char *q1 = strchr(q0 + 1, '"');
        if (!q1) continue;
        Choice c;
        if (sscanf(q1 + 1, " : {\"variant\": %d, \"proposals\": %ld, \"ns_per_proposal\": %lf", &c.variant,
                   &c.proposals, &c.ns) == 3)
            m[std::string(q0 + 1, q1)] = c;
    }
    fclose(f);
    return m;
}

int write_cache(tn_ctx *ctx, const char *path, const std::map<std::string, Choice> &m) {
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return tn_fail(ctx, TN_EINVAL, std::string("cannot write the tuning cache ") + tmp);
    fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : m)
        fprintf(f, "  \"%s\": {\"variant\": %d, \"proposals\": %ld, \"ns_per_proposal\": %.4f}%s\n",
                kv.first.c_str(), kv.second.variant, kv.second.proposals, kv.second.ns,
                ++i < m.size() ? "," : "");
    fprintf(f, "}\n");
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), path) != 0) {
        (void)remove(tmp.c_str());
        return tn_fail(ctx, TN_EINVAL, std::string("cannot write the tuning cache ") + path);
    }
    return TN_OK;
}

// Counters (clamps, near-threshold draws, ...) are the user's statistics: the
// timing launches must leave them as they were.
struct CounterGuard {
    tn_ctx *ctx;
    unsigned long long saved[CNT_N];
    bool ok = false;
    explicit CounterGuard(tn_ctx *c) : ctx(c) {
        ok = hipMemcpy(saved, ctx->counters, sizeof saved, hipMemcpyDeviceToHost) == hipSuccess;
    }
    int restore() {
        if (!ok) return tn_fail(ctx, TN_EHIP, "cannot read the counters");
        TN_HIP(ctx, hipMemcpy(ctx->counters, saved, sizeof saved, hipMemcpyHostToDevice));
        return TN_OK;
    }
};

// Mean milliseconds of one launch of `launch`, after one untimed launch; the
// number of timed launches adapts to give about 50 ms of work.
template <class F>
int time_launches(tn_ctx *ctx, F launch, double *ms_out) {
    hipEvent_t e0, e1;
    TN_HIP(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return tn_fail(ctx, TN_EHIP, "hipEventCreate failed");
    }
    int rc = TN_OK;
    float ms = 0.0f;
    int reps = 1;
    for (int pass = 0; pass < 2 && rc == TN_OK; ++pass) {
        // pass 0: one launch (warm-up and estimate); pass 1: the measurement
        if (hipEventRecord(e0, ctx->stream) != hipSuccess) rc = tn_fail(ctx, TN_EHIP, "hipEventRecord failed");
        for (int i = 0; i < reps && rc == TN_OK; ++i) rc = launch(i);
        if (rc == TN_OK && (hipEventRecord(e1, ctx->stream) != hipSuccess ||
                            hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = tn_fail(ctx, TN_EHIP, "timing the sampler failed");
        if (pass == 0) reps = std::max(1, std::min(8, (int)(50.0 / std::max(ms, 1e-3f))));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == TN_OK) *ms_out = ms / reps;
    return rc;
}

bool better(double ns, double best_ns) { return ns < 0.99 * best_ns; }   // ties: the earlier candidate

}  // namespace

extern "C" {

int tn_autotune(tn_ctx *ctx, int chains, int max_steps, const char *cache_path, int *variant_out,
                int *steps_out) {
    (void)hipGetLastError();
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    if (!ctx->has_env) return tn_fail(ctx, TN_ESTATE, "no environment: build or set one first");
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "cannot time kernels during graph capture");
    if (ctx->qd) return tn_fail(ctx, TN_EINVAL, "not available for a Potts context (tn_potts_build_env)");
    if (chains < 1 || max_steps < 1) return tn_fail(ctx, TN_EINVAL, "chains < 1 or max_steps < 1");
    if (max_steps > 64) max_steps = 64;
    const int NT = ctx->Dp / 16;
    const bool plain = ctx->prec == TN_FP64;
    const std::string key = arch_name(ctx->device) + "|" + std::to_string(ctx->Lx) + "x" +
                            std::to_string(ctx->Ly) + "|D" + std::to_string(ctx->D) + "|" +
                            prec_name(ctx->prec) + "|chains" + std::to_string(chains) + "|steps" +
                            std::to_string(max_steps);
    std::map<std::string, Choice> cache;
    if (cache_path) cache = read_cache(cache_path);
    Choice best;
    auto hit = cache.find(key);
    const int nvar = (plain || ctx->prec == TN_FP64_MFMA) ? 1 : tn_team_variants(NT, ctx->prec == TN_BF16);
    if (hit != cache.end() && hit->second.variant >= 0 && hit->second.variant < nvar &&
        hit->second.proposals >= 1) {
        best = hit->second;
    } else {
        // candidate step counts: powers of two up to max_steps, and max_steps;
        // at most a quarter of the free device memory for buffers and scratch
        size_t free_b = 0, total_b = 0;
        TN_HIP(ctx, hipMemGetInfo(&free_b, &total_b));
        const size_t nsite = (size_t)ctx->Lx * ctx->Ly;
        const size_t per_prop = nsite + 2 * sizeof(double) +
                                (plain ? (size_t)ctx->Lx * 2 * ctx->D * sizeof(double)
                                       : (size_t)ctx->Lx * 2 * ctx->Dp * sizeof(float));
        std::vector<int> steps;
        for (int m = 1; m <= max_steps; m *= 2) steps.push_back(m);
        if (steps.back() != max_steps) steps.push_back(max_steps);
        std::vector<int> fit;
        for (int m : steps)
            if ((size_t)m * chains <= (size_t)INT32_MAX / 2 && (size_t)m * chains * per_prop <= free_b / 4)
                fit.push_back(m);
        if (fit.empty()) return tn_fail(ctx, TN_ENOMEM, "not enough device memory for one step's proposals");
        // the launches timed: every candidate count and the remainder it
        // leaves of max_steps (the last launch of a run of max_steps steps)
        std::vector<int> timed(fit);
        for (int m : fit)
            if (max_steps % m) timed.push_back(max_steps % m);
        std::sort(timed.begin(), timed.end());
        timed.erase(std::unique(timed.begin(), timed.end()), timed.end());
        const int mmax = fit.back();
        const size_t spin_bytes = (((size_t)mmax * chains * nsite + 255) / 256) * 256;
        const size_t need = spin_bytes + 2 * (size_t)mmax * chains * sizeof(double);
        int rc;
        if (need > ctx->pcap) {
            void *p = ctx->pspins;
            if ((rc = tn_ensure(ctx, &p, &ctx->pcap, need))) return rc;
            ctx->pspins = (int8_t *)p;
        }
        int8_t *S = ctx->pspins;
        double *lq = (double *)(ctx->pspins + spin_bytes);
        double *E = lq + (size_t)mmax * chains;
        CounterGuard guard(ctx);
        std::map<std::pair<int, int>, double> T;   // (variant, steps per launch) -> ms per launch
        for (int m : timed)
            for (int v = 0; v < nvar; ++v) {
                const int batch = m * chains;
                double ms = 0.0;
                rc = time_launches(ctx, [&](int i) {
                        return plain ? tn_run_fp64(ctx, batch, 0x7475ull, (uint64_t)i * m, chains, 0, S, false, lq, E)
                                     : tn_run_mfma(ctx, batch, 0x7475ull, (uint64_t)i * m, chains, 0, S, false, lq, E, v);
                    }, &ms);
                if (rc) {
                    (void)guard.restore();
                    return rc;
                }
                T[{v, m}] = ms;
            }
        // the fastest run of max_steps steps: launches of m steps and one of
        // the remainder, all in the same variant (as tn_mh_run draws them)
        best.ns = -1.0;
        for (int m : fit)
            for (int v = 0; v < nvar; ++v) {
                const int q = max_steps / m, r = max_steps % m;
                const double total = q * T[{v, m}] + (r ? T[{v, r}] : 0.0);
                const double ns = total * 1e6 / ((double)max_steps * chains);
                if (best.ns < 0.0 || better(ns, best.ns)) {
                    best.variant = v;
                    best.proposals = (long)m * chains;
                    best.ns = ns;
                }
            }
        if ((rc = guard.restore())) return rc;
        if (cache_path) {
            cache = read_cache(cache_path);   // another process may have added entries meanwhile
            cache[key] = best;
            if ((rc = write_cache(ctx, cache_path, cache))) return rc;
        }
    }
    tn_tuned &t = ctx->tuned;
    t.valid = true;
    t.Lx = ctx->Lx;
    t.Ly = ctx->Ly;
    t.Dp = ctx->Dp;
    t.prec = ctx->prec;
    t.variant = best.variant;
    t.proposals = best.proposals;
    if (variant_out) *variant_out = best.variant;
    if (steps_out) *steps_out = (int)std::max(1L, (best.proposals + chains - 1) / chains);
    return TN_OK;
}

int tn_autotune_multi(tn_ctx *ctx, const char *cache_path, int *variants_out) {
    (void)hipGetLastError();
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    if (!ctx->has_multi) return tn_fail(ctx, TN_ESTATE, "no instances: call tn_build_env_multi first");
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "cannot time kernels during graph capture");
    int rc;
    if ((rc = tn_multi_prepare(ctx))) return rc;
    std::vector<tn_samp_desc> sd;
    std::vector<tn_multi_group> groups;
    tn_multi_groups(ctx, sd, groups);
    if (variants_out)
        for (int i = 0; i < 8; ++i) variants_out[i] = -1;
    if (groups.empty()) return TN_OK;
    std::map<std::string, Choice> cache;
    if (cache_path) cache = read_cache(cache_path);
    bool dirty = false;
    void *dd = nullptr;
    TN_HIP(ctx, hipMalloc(&dd, sd.size() * sizeof(tn_samp_desc)));
    if (hipMemcpy(dd, sd.data(), sd.size() * sizeof(tn_samp_desc), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dd);
        return tn_fail(ctx, TN_EHIP, "cannot upload the sampler descriptors");
    }
    const tn_samp_desc *sdev = (const tn_samp_desc *)dd;
    const std::string arch = arch_name(ctx->device);
    for (const tn_multi_group &g : groups) {
        // the key lists the group's instances as (lattice, D, chains) x count
        // (the group's instances, selected as tn_multi_groups does)
        std::map<std::string, int> shapes;
        long props = 0;
        for (size_t i = 0; i < ctx->kids.size(); ++i) {
            const tn_ctx *k = ctx->kids[i];
            const int C = ctx->kid_chains[i];
            if (k->prec == TN_FP64 || C == 0 || k->Dp / 16 != g.NT || (k->prec == TN_BF16) != g.bf16) continue;
            ++shapes[std::to_string(k->Lx) + "x" + std::to_string(k->Ly) + ":D" + std::to_string(k->D) + ":c" +
                     std::to_string(C)];
            props += C;
        }
        std::string key = arch + "|multi|" + (g.bf16 ? "bf16" : "fp32") + "|NT" + std::to_string(g.NT) + "|";
        bool first = true;
        for (const auto &kv : shapes) {
            key += (first ? "" : ",") + kv.first + "*" + std::to_string(kv.second);
            first = false;
        }
        const int nvar = tn_team_variants(g.NT, g.bf16);
        Choice best;
        auto hit = cache.find(key);
        if (hit != cache.end() && hit->second.variant >= 0 && hit->second.variant < nvar) {
            best = hit->second;
        } else {
            std::vector<CounterGuard> guards;
            for (tn_ctx *k : ctx->kids) guards.emplace_back(k);
            best.ns = -1.0;
            for (int v = 0; v < nvar && rc == TN_OK; ++v) {
                double ms = 0.0;
                rc = time_launches(ctx, [&](int i) {
                        return tn_run_mfma_multi(ctx, g.NT, g.bf16, v, sdev + g.first, g.count, g.blocks,
                                                 g.maxLx, 0x7475ull, (uint64_t)i);
                    }, &ms);
                if (rc == TN_OK) {
                    const double ns = ms * 1e6 / (double)props;
                    if (best.ns < 0.0 || better(ns, best.ns)) {
                        best.variant = v;
                        best.proposals = props;
                        best.ns = ns;
                    }
                }
            }
            for (CounterGuard &q : guards) {
                const int r2 = q.restore();
                if (rc == TN_OK && r2) rc = tn_fail(ctx, r2, q.ctx->err);
            }
            if (rc) break;
            cache[key] = best;
            dirty = true;
        }
        ctx->multi_variant[g.bf16 ? 1 : 0][g.NT] = best.variant;
        if (variants_out) variants_out[(g.bf16 ? 4 : 0) + g.NT - 1] = best.variant;
    }
    (void)hipFree(dd);
    if (rc) return rc;
    if (cache_path && dirty) {
        std::map<std::string, Choice> merged = read_cache(cache_path);
        for (const auto &kv : cache) merged[kv.first] = kv.second;
        if ((rc = write_cache(ctx, cache_path, merged))) return rc;
    }
    return TN_OK;
}

}  // extern "C"
