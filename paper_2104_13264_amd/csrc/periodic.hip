// Periodic boundaries by alternately frozen lines (Section "Arbitrary boundary
// conditions"): a lattice whose opposite edges are identified is sampled with
// the open-boundary sampler by keeping one line of spins (a column on a
// cylinder along x, a row on one along y, a cross on a torus) fixed during a
// TNMH step.  The free spins form an open lattice in which a site next to the
// frozen line feels the field J s_frozen of that bond; the frozen line moves
// between steps so that every spin is refreshed.
//
// Each chain's open model depends on its own frozen spins, so a step builds
// one environment stack per chain.  A step is:
//   k_cut      per chain: the open lattice's spins and fields, per instance:
//              its open couplings (the site map and field order of tnmh.h)
//   row steps  the batched environment build of every chain (env_build.hip)
//   status     top overlaps and each build's outcome, one copy to the host
//   operands   the sampler operands of every chain, one batched launch pair
//              (operands.hip)
//   eval       ln q and E of the current free spins under the new cut
//   sample     one proposal per chain (id j, instance m)
//   accept     Eq. (mh-acc) per chain with the open model's ln q and energies
//   k_uncut    the free spins written back, periodic energies, accept flags
#include "common.hpp"

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#pragma clang fp contract(off)

namespace {

// One periodic instance as the cut kernels see it (device copy).
struct tn_per_desc {
    const double *Jh, *Jv, *h;   // periodic couplings and field (h may be NULL)
    double *Jho, *Jvo;           // open couplings under the current cut
    int first, chains;
    double beta;
};

struct tn_periodic {
    int Lx = 0, Ly = 0, wx = 0, wy = 0, D = 0, prec = 0, n = 0, total = 0;
    int Lxo = 0, Lyo = 0, nso = 0;
    std::vector<int> first, chains;
    std::vector<double> beta;
    std::vector<tn_ctx *> kids;   // one per chain: its open model and environments
    void *arena = nullptr;        // every device buffer below
    tn_per_desc *pd = nullptr;    // [n]
    int *inst_of = nullptr;       // [total]
    double *ho = nullptr;         // [total][nso] open fields
    int8_t *os = nullptr;         // [total][nso] current free spins
    int8_t *ps = nullptr;         // [total][nso] proposals
    double *slogq = nullptr, *sE = nullptr, *plogq = nullptr, *pE = nullptr;   // [total]
    uint8_t *acc = nullptr;       // [total]
    int *status = nullptr;        // [total]
    float *gscr = nullptr;        // batched-sampler scratch, gscr_per floats per chain
    size_t gscr_per = 0;
    tn_samp_desc *sd_eval = nullptr, *sd_samp = nullptr;   // [total] each
    tn_acc_desc *ad = nullptr;    // [instances with chains]
    tn_ops_desc *od = nullptr;    // [total]: every chain's operand build
    int nacc = 0;
    bool descs_ready = false, ops_ready = false;
    tn_build_plan plan;
    std::vector<int> hstatus;
};

constexpr int PT_THREADS = 256;

__global__ void __launch_bounds__(PT_THREADS)
k_cut(const tn_per_desc *__restrict__ pd, const int *__restrict__ inst_of, int Lx, int Ly, int wx, int wy,
      int Lxo, int Lyo, int cr, int cc, const int8_t *__restrict__ S, int8_t *__restrict__ os,
      double *__restrict__ ho) {
    const int g = blockIdx.x;
    const tn_per_desc P = pd[inst_of[g]];
    const int nso = Lxo * Lyo;
    const int JhW = wx ? Lx : Lx - 1;
    const int8_t *s = S + (size_t)g * Lx * Ly;
    for (int i = threadIdx.x; i < nso; i += PT_THREADS) {
        const int ro = i / Lxo, co = i - ro * Lxo;
        const int r = wy ? (cr + 1 + ro) % Ly : ro;
        const int c = wx ? (cc + 1 + co) % Lx : co;
        os[(size_t)g * nso + i] = s[r * Lx + c];
        const double base = P.h ? P.h[r * Lx + c] : 0.0;
        const double fl = (wx && co == 0) ? P.Jh[r * JhW + cc] * (double)s[r * Lx + cc] : 0.0;
        const double fr = (wx && co == Lxo - 1) ? P.Jh[r * JhW + (cc + Lx - 1) % Lx] * (double)s[r * Lx + cc] : 0.0;
        const double fu = (wy && ro == 0) ? P.Jv[cr * Lx + c] * (double)s[cr * Lx + c] : 0.0;
        const double fd = (wy && ro == Lyo - 1) ? P.Jv[((cr + Ly - 1) % Ly) * Lx + c] * (double)s[cr * Lx + c] : 0.0;
        ho[(size_t)g * nso + i] = (((base + fl) + fr) + fu) + fd;
    }
    if (g == P.first) {   // the instance's open couplings, shared by its chains
        for (int i = threadIdx.x; i < Lyo * (Lxo - 1); i += PT_THREADS) {
            const int ro = i / (Lxo - 1), co = i - ro * (Lxo - 1);
            const int r = wy ? (cr + 1 + ro) % Ly : ro;
            const int c = wx ? (cc + 1 + co) % Lx : co;
            P.Jho[i] = P.Jh[r * JhW + c];
        }
        for (int i = threadIdx.x; i < (Lyo - 1) * Lxo; i += PT_THREADS) {
            const int ro = i / Lxo, co = i - ro * Lxo;
            const int r = wy ? (cr + 1 + ro) % Ly : ro;
            const int c = wx ? (cc + 1 + co) % Lx : co;
            P.Jvo[i] = P.Jv[r * Lx + c];
        }
    }
}

// Writes the free spins back (os != NULL) and the periodic energy of every
// chain, and copies the accept flags (acc != NULL).
__global__ void __launch_bounds__(PT_THREADS)
k_uncut(const tn_per_desc *__restrict__ pd, const int *__restrict__ inst_of, int Lx, int Ly, int wx, int wy,
        int Lxo, int Lyo, int cr, int cc, const int8_t *__restrict__ os, int8_t *__restrict__ S,
        double *__restrict__ energy, const uint8_t *__restrict__ acc, uint8_t *__restrict__ accepted) {
    extern __shared__ int8_t sp[];   // [Ly][Lx]
    __shared__ double red[PT_THREADS / 64];
    const int g = blockIdx.x;
    const tn_per_desc P = pd[inst_of[g]];
    const int N = Lx * Ly, nso = Lxo * Lyo;
    const int JhW = wx ? Lx : Lx - 1;
    int8_t *s = S + (size_t)g * N;
    for (int i = threadIdx.x; i < N; i += PT_THREADS) sp[i] = s[i];
    __syncthreads();
    if (os) {
        for (int i = threadIdx.x; i < nso; i += PT_THREADS) {
            const int ro = i / Lxo, co = i - ro * Lxo;
            const int r = wy ? (cr + 1 + ro) % Ly : ro;
            const int c = wx ? (cc + 1 + co) % Lx : co;
            sp[r * Lx + c] = os[(size_t)g * nso + i];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < N; i += PT_THREADS) s[i] = sp[i];
    }
    double e = 0.0;
    for (int i = threadIdx.x; i < N; i += PT_THREADS) {
        const int r = i / Lx, c = i - r * Lx;
        const double si = (double)sp[i];
        double t = P.h ? P.h[i] * si : 0.0;
        if (wx || c + 1 < Lx) t = t + P.Jh[r * JhW + c] * (si * (double)sp[r * Lx + (c + 1) % Lx]);
        if (wy || r + 1 < Ly) t = t + P.Jv[r * Lx + c] * (si * (double)sp[((r + 1) % Ly) * Lx + c]);
        e = e - t;
    }
    e = tn_block_sum(e, red);
    if (threadIdx.x == 0) {
        energy[g] = e;
        if (acc) accepted[g] = acc[g];
    }
}

// Checkerboard Metropolis sweeps on the identified lattice (Sec. 3: single
// spin flips between TNMH steps), one workgroup per chain with its spins in
// LDS.  Local field h + left + right + up + down with the wrapping
// neighbours, in that order; flip iff u < exp(-(beta 2 s F)); u is word i % 4
// of Philox stream 2 at counter (sweep * 2^14 + i / 4, chain j, step,
// instance m << 2 | 2).  Wrapped lengths are even, so same-colour sites share
// no bond.
__global__ void __launch_bounds__(PT_THREADS)
k_per_metropolis(const tn_per_desc *__restrict__ pd, const int *__restrict__ inst_of, int Lx, int Ly, int wx,
                 int wy, int nsweeps, int8_t *__restrict__ S, uint32_t k0, uint32_t k1, uint32_t step,
                 unsigned long long *__restrict__ counters) {
    extern __shared__ int8_t sp[];   // [Ly][Lx]
    const int g = blockIdx.x;
    const int m = inst_of[g];
    const tn_per_desc P = pd[m];
    const uint32_t j = (uint32_t)(g - P.first);
    const int N = Lx * Ly, JhW = wx ? Lx : Lx - 1;
    int8_t *s = S + (size_t)g * N;
    for (int i = threadIdx.x; i < N; i += PT_THREADS) sp[i] = s[i];
    __syncthreads();
    uint32_t flips = 0;
    const int nblk = (N + 3) >> 2;
    for (int k = 0; k < nsweeps; ++k) {
        for (int colour = 0; colour < 2; ++colour) {
            for (int b = threadIdx.x; b < nblk; b += PT_THREADS) {
                const uint4 w = tn_philox(make_uint4(((uint32_t)k << 14) | (uint32_t)b, j, step,
                                                     ((uint32_t)m << 2) | 2u),
                                          k0, k1);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = 4 * b + q;
                    if (i >= N) break;
                    const int r = i / Lx, c = i - r * Lx;
                    if (((r + c) & 1) != colour) continue;
                    const int cl = c > 0 ? c - 1 : Lx - 1, cr = c + 1 < Lx ? c + 1 : 0;
                    const int ru = r > 0 ? r - 1 : Ly - 1, rd = r + 1 < Ly ? r + 1 : 0;
                    double F = P.h ? P.h[i] : 0.0;
                    if (c > 0 || wx) F = F + P.Jh[r * JhW + cl] * (double)sp[r * Lx + cl];
                    if (c + 1 < Lx || wx) F = F + P.Jh[r * JhW + c] * (double)sp[r * Lx + cr];
                    if (r > 0 || wy) F = F + P.Jv[ru * Lx + c] * (double)sp[ru * Lx + c];
                    if (r + 1 < Ly || wy) F = F + P.Jv[r * Lx + c] * (double)sp[rd * Lx + c];
                    const double dE = (2.0 * (double)sp[i]) * F;
                    if (tn_u01(tn_word(w, q)) < exp(-(P.beta * dE))) {
                        sp[i] = (int8_t)(-sp[i]);
                        ++flips;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < N; i += PT_THREADS) s[i] = sp[i];
    if (flips) atomicAdd(&counters[CNT_FLIPS], (unsigned long long)flips);
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

tn_periodic *per_of(tn_ctx *ctx) { return (tn_periodic *)ctx->per; }

int need_periodic(tn_ctx *ctx) {
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    if (!ctx->per) return tn_fail(ctx, TN_ESTATE, "no periodic lattice: call tn_periodic_setup first");
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "not allowed while capturing a graph");
    return TN_OK;
}

// The device descriptors of the samplers and the acceptance: fixed once the
// operands exist (every pointer in them stays put from step to step).
int make_descs(tn_ctx *ctx, tn_periodic *P) {
    std::vector<tn_samp_desc> ev(P->total), sa(P->total);
    std::vector<tn_acc_desc> ac;
    for (int m = 0; m < P->n; ++m) {
        for (int j = 0; j < P->chains[m]; ++j) {
            const int g = P->first[m] + j;
            tn_ctx *k = P->kids[g];
            float *gs = P->gscr + (size_t)g * P->gscr_per;
            ev[g] = tn_samp_desc_of(k, 1, P->os + (size_t)g * P->nso, P->slogq + g, P->sE + g, gs, 1, (uint64_t)j);
            sa[g] = tn_samp_desc_of(k, 1, P->ps + (size_t)g * P->nso, P->plogq + g, P->pE + g, gs, 1, (uint64_t)j);
            ev[g].blk0 = sa[g].blk0 = 8 * g;   // one team of eight 16-proposal units per chain
            ev[g].counters = sa[g].counters = ctx->counters;
        }
        if (P->chains[m] == 0) continue;
        tn_acc_desc A;
        const int f = P->first[m];
        A.chains = P->chains[m];
        A.nsite = P->nso;
        A.beta = P->beta[m];
        A.inst = (uint32_t)m;
        A.blk0 = f;
        A.pspins = P->ps + (size_t)f * P->nso;
        A.plogq = P->plogq + f;
        A.pE = P->pE + f;
        A.sspins = P->os + (size_t)f * P->nso;
        A.slogq = P->slogq + f;
        A.sE = P->sE + f;
        A.accepted = P->acc + f;
        A.counters = ctx->counters;
        A.eser = nullptr;
        ac.push_back(A);
    }
    TN_HIP(ctx, hipMemcpy(P->sd_eval, ev.data(), ev.size() * sizeof(tn_samp_desc), hipMemcpyHostToDevice));
    TN_HIP(ctx, hipMemcpy(P->sd_samp, sa.data(), sa.size() * sizeof(tn_samp_desc), hipMemcpyHostToDevice));
    TN_HIP(ctx, hipMemcpy(P->ad, ac.data(), ac.size() * sizeof(tn_acc_desc), hipMemcpyHostToDevice));
    P->nacc = (int)ac.size();
    P->descs_ready = true;
    return TN_OK;
}

}  // namespace

void tn_periodic_free(tn_ctx *ctx) {
    tn_periodic *P = per_of(ctx);
    if (!P) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (tn_ctx *k : P->kids) {
        // borrowed: couplings, fields and the small buffers carved from the arena
        k->Jh = k->Jv = k->h = nullptr;
        k->counters = nullptr;
        k->scal = nullptr;
        k->dims = nullptr;
        k->ell = nullptr;
        k->cst = nullptr;
        k->xdims = nullptr;
        k->dstep = nullptr;
        tn_free_ctx(k);
        delete k;
    }
    if (P->arena) (void)hipFree(P->arena);
    delete P;
    ctx->per = nullptr;
}

extern "C" {

int tn_periodic_setup(tn_ctx *ctx, int Lx, int Ly, int wrap_x, int wrap_y, int D, int prec, int n,
                      const tn_periodic_instance *inst) {
    (void)hipGetLastError();
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "not allowed while capturing a graph");
    const int wx = wrap_x ? 1 : 0, wy = wrap_y ? 1 : 0;
    if (Lx < 1 || Ly < 1) return tn_fail(ctx, TN_EINVAL, "Lx and Ly must be >= 1");
    if ((wx && Lx < 3) || (wy && Ly < 3))
        return tn_fail(ctx, TN_EINVAL, "a wrapped direction needs at least 3 sites");
    if ((long)Lx * Ly > 65536) return tn_fail(ctx, TN_EINVAL, "more than 65536 sites");
    const int Lxo = Lx - wx, Lyo = Ly - wy;
    if (Lxo > 256) return tn_fail(ctx, TN_EINVAL, "open lattice wider than 256 columns");
    if (D < 1 || D > TN_MAX_D) return tn_fail(ctx, TN_EINVAL, "D must be in 1..64");
    if (prec != TN_FP64 && prec != TN_FP32 && prec != TN_BF16)
        return tn_fail(ctx, TN_EINVAL, "prec must be TN_FP64, TN_FP32 or TN_BF16");
    if (n < 1 || !inst) return tn_fail(ctx, TN_EINVAL, "need n >= 1 instances");
    long total = 0;
    for (int m = 0; m < n; ++m) {
        if (inst[m].chains < 0) return tn_fail(ctx, TN_EINVAL, "chains < 0");
        if (!std::isfinite(inst[m].beta)) return tn_fail(ctx, TN_EINVAL, "beta must be finite");
        if ((Ly * (Lx - 1 + wx) > 0 && !inst[m].Jh) || ((Ly - 1 + wy) * Lx > 0 && !inst[m].Jv))
            return tn_fail(ctx, TN_EINVAL, "instance " + std::to_string(m) + ": NULL couplings");
        total += inst[m].chains;
    }
    if (total < 1) return tn_fail(ctx, TN_EINVAL, "no chains");
    if (total > (1 << 20)) return tn_fail(ctx, TN_EINVAL, "more than 2^20 chains");
    tn_periodic_free(ctx);
    tn_periodic *P = new (std::nothrow) tn_periodic();
    if (!P) return tn_fail(ctx, TN_ENOMEM, "out of host memory");
    ctx->per = P;
    P->Lx = Lx;
    P->Ly = Ly;
    P->wx = wx;
    P->wy = wy;
    P->D = D;
    P->prec = prec;
    P->n = n;
    P->total = (int)total;
    P->Lxo = Lxo;
    P->Lyo = Lyo;
    P->nso = Lxo * Lyo;
    const int T = P->total, nso = P->nso;
    const size_t nh = (size_t)Ly * (Lx - 1 + wx), nv = (size_t)(Ly - 1 + wy) * Lx, nf = (size_t)Lx * Ly;
    const size_t nho = (size_t)Lyo * (Lxo - 1), nvo = (size_t)(Lyo - 1) * Lxo;
    const int Dp = ((D + 15) / 16) * 16;
    // per-chain small buffers: counters, scalars, bond dims, log-normalisers,
    // truncation columns and the build's dimension scratch
    const size_t b_cnt = align256(CNT_N * sizeof(unsigned long long)), b_scal = align256(16 * sizeof(double));
    const size_t b_dims = align256((size_t)(Lyo + 1) * (Lxo + 1) * sizeof(int));
    const size_t b_ell = align256((size_t)(Lyo + 1) * sizeof(double));
    const size_t b_cst = align256((size_t)(Lyo + 1) * sizeof(int));
    const size_t b_xd = align256(2 * (4 * TN_MAX_D + 1) * sizeof(int) + 2 * 1024 * sizeof(int));
    const size_t small = b_cnt + b_scal + b_dims + b_ell + b_cst + b_xd;
    P->gscr_per = (size_t)8 * Lxo * 2 * Dp * 16;   // floats: one team of eight units, as the batched sampler
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes ? bytes : 1);
        return o;
    };
    const size_t o_pd = take(n * sizeof(tn_per_desc)), o_inst = take(T * sizeof(int));
    const size_t o_Jt = take((size_t)n * (nh + nv + nf) * sizeof(double));
    const size_t o_Jo = take((size_t)n * (nho + nvo) * sizeof(double));
    const size_t o_ho = take((size_t)T * nso * sizeof(double));
    const size_t o_os = take((size_t)T * nso), o_ps = take((size_t)T * nso);
    const size_t o_q = take((size_t)4 * T * sizeof(double)), o_acc = take(T), o_st = take(T * sizeof(int));
    const size_t o_gs = prec == TN_FP64 ? take(0) : take((size_t)T * P->gscr_per * sizeof(float));
    const size_t o_sd = take((size_t)2 * T * sizeof(tn_samp_desc)), o_ad = take((size_t)n * sizeof(tn_acc_desc));
    const size_t o_od = take((size_t)T * sizeof(tn_ops_desc));
    const size_t o_small = take((size_t)T * small);
    if (hipMalloc(&P->arena, off) != hipSuccess) {
        (void)hipGetLastError();
        P->arena = nullptr;
        tn_periodic_free(ctx);
        return tn_fail(ctx, TN_ENOMEM, "device allocation of " + std::to_string(off) + " bytes failed");
    }
    unsigned char *A = (unsigned char *)P->arena;
    P->pd = (tn_per_desc *)(A + o_pd);
    P->inst_of = (int *)(A + o_inst);
    double *Jt = (double *)(A + o_Jt), *Jo = (double *)(A + o_Jo);
    P->ho = (double *)(A + o_ho);
    P->os = (int8_t *)(A + o_os);
    P->ps = (int8_t *)(A + o_ps);
    P->slogq = (double *)(A + o_q);
    P->sE = P->slogq + T;
    P->plogq = P->sE + T;
    P->pE = P->plogq + T;
    P->acc = A + o_acc;
    P->status = (int *)(A + o_st);
    P->gscr = prec == TN_FP64 ? nullptr : (float *)(A + o_gs);
    P->sd_eval = (tn_samp_desc *)(A + o_sd);
    P->sd_samp = P->sd_eval + T;
    P->ad = (tn_acc_desc *)(A + o_ad);
    P->od = (tn_ops_desc *)(A + o_od);
    int rc = TN_OK;
    auto bail = [&](int code, const std::string &msg) {
        tn_periodic_free(ctx);
        return tn_fail(ctx, code, msg);
    };
    if (hipMemsetAsync(A + o_small, 0, (size_t)T * small, ctx->stream) != hipSuccess)
        return bail(TN_EHIP, "clearing the chain buffers failed");
    std::vector<tn_per_desc> pd(n);
    std::vector<int> inst_of(T);
    P->first.assign(n, 0);
    P->chains.assign(n, 0);
    P->beta.assign(n, 0.0);
    int g = 0;
    for (int m = 0; m < n; ++m) {
        double *Jh = Jt + (size_t)m * (nh + nv + nf), *Jv = Jh + nh, *h = Jv + nv;
        if (nh && hipMemcpyAsync(Jh, inst[m].Jh, nh * sizeof(double), hipMemcpyDefault, ctx->stream) != hipSuccess)
            return bail(TN_EHIP, "coupling copy failed");
        if (nv && hipMemcpyAsync(Jv, inst[m].Jv, nv * sizeof(double), hipMemcpyDefault, ctx->stream) != hipSuccess)
            return bail(TN_EHIP, "coupling copy failed");
        if (inst[m].h && hipMemcpyAsync(h, inst[m].h, nf * sizeof(double), hipMemcpyDefault, ctx->stream) != hipSuccess)
            return bail(TN_EHIP, "field copy failed");
        pd[m].Jh = Jh;
        pd[m].Jv = Jv;
        pd[m].h = inst[m].h ? h : nullptr;
        pd[m].Jho = Jo + (size_t)m * (nho + nvo);
        pd[m].Jvo = pd[m].Jho + nho;
        pd[m].first = g;
        pd[m].chains = inst[m].chains;
        pd[m].beta = inst[m].beta;
        P->first[m] = g;
        P->chains[m] = inst[m].chains;
        P->beta[m] = inst[m].beta;
        for (int j = 0; j < inst[m].chains; ++j, ++g) {
            inst_of[g] = m;
            tn_ctx *k = new (std::nothrow) tn_ctx();
            if (!k) return bail(TN_ENOMEM, "out of host memory");
            P->kids.push_back(k);
            unsigned char *sm = A + o_small + (size_t)g * small;
            k->stream = ctx->stream;
            k->device = ctx->device;
            k->dstep = ctx->dstep;
            k->own_dstep = false;
            k->counters = (unsigned long long *)sm;
            k->scal = (double *)(sm + b_cnt);
            k->dims = (int *)(sm + b_cnt + b_scal);
            k->ell = (double *)(sm + b_cnt + b_scal + b_dims);
            k->cst = (int *)(sm + b_cnt + b_scal + b_dims + b_ell);
            k->xdims = (int *)(sm + b_cnt + b_scal + b_dims + b_ell + b_cst);
            k->Lx = Lxo;
            k->Ly = Lyo;
            k->D = D;
            k->Dp = Dp;
            k->beta = inst[m].beta;
            k->prec = prec;
            k->fit_sweeps = ctx->fit_sweeps;
            k->inst = m;
            k->Jh = pd[m].Jho;
            k->Jv = pd[m].Jvo;
            k->h = P->ho + (size_t)g * nso;
            const size_t envn = (size_t)(Lyo + 1) * Lxo * 2 * D * D;
            if ((rc = tn_ensure(k, (void **)&k->env, &k->env_cap, envn * sizeof(double))))
                return bail(rc, k->err);
        }
    }
    if (hipMemcpy(P->pd, pd.data(), n * sizeof(tn_per_desc), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P->inst_of, inst_of.data(), T * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return bail(TN_EHIP, "descriptor copy failed");
    std::string e;
    if ((rc = tn_env_build_prepare(P->kids.data(), T, ctx->stream, &e, &P->plan))) return bail(rc, e);
    P->hstatus.assign(T, 0);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return bail(TN_EHIP, "set-up failed");
    return TN_OK;
}

int tn_periodic_step(tn_ctx *ctx, uint64_t seed, uint64_t step, int cut_row, int cut_col, int8_t *spins,
                     double *energy, uint8_t *accepted) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_periodic(ctx))) return rc;
    tn_periodic *P = per_of(ctx);
    if (!spins || !energy || !accepted) return tn_fail(ctx, TN_EINVAL, "NULL buffer");
    if (P->wy && (cut_row < 0 || cut_row >= P->Ly)) return tn_fail(ctx, TN_EINVAL, "cut_row out of range");
    if (P->wx && (cut_col < 0 || cut_col >= P->Lx)) return tn_fail(ctx, TN_EINVAL, "cut_col out of range");
    const int cr = P->wy ? cut_row : 0, cc = P->wx ? cut_col : 0;
    const int T = P->total;
    hipLaunchKernelGGL(k_cut, dim3(T), dim3(PT_THREADS), 0, ctx->stream, P->pd, P->inst_of, P->Lx, P->Ly, P->wx,
                       P->wy, P->Lxo, P->Lyo, cr, cc, spins, P->os, P->ho);
    TN_HIP(ctx, hipGetLastError());
    std::string e;
    if ((rc = tn_env_build_steps(&P->plan, 0, P->plan.maxLy - 1, ctx->stream, &e))) return tn_fail(ctx, rc, e);
    if ((rc = tn_env_build_top_status(&P->plan, P->status, ctx->stream)))
        return tn_fail(ctx, rc, "top overlap launch failed");
    TN_HIP(ctx, hipMemcpy(P->hstatus.data(), P->status, T * sizeof(int), hipMemcpyDeviceToHost));
    for (int g = 0; g < T; ++g)
        if (P->hstatus[g])
            return tn_fail(ctx, P->hstatus[g] == 2 ? TN_ENOCONV : TN_ENONPOS,
                           std::string(P->hstatus[g] == 2 ? "Jacobi SVD did not converge"
                                                          : "approximate partition function is not positive") +
                               " for chain " + std::to_string(g) + " under this cut");
    if (!P->ops_ready) {   // first step: allocates every chain's operand buffers
        std::vector<tn_ops_desc> od(T);
        for (int g = 0; g < T; ++g) {
            if ((rc = tn_make_operands(P->kids[g], P->prec))) return tn_fail(ctx, rc, P->kids[g]->err);
            od[g] = tn_ops_desc_of(P->kids[g], P->prec);
        }
        TN_HIP(ctx, hipMemcpy(P->od, od.data(), T * sizeof(tn_ops_desc), hipMemcpyHostToDevice));
        P->ops_ready = true;
    } else if ((rc = tn_make_operands_many(ctx, P->od, T, P->Lxo, P->Lyo, ((P->D + 15) / 16) * 16))) {
        return rc;
    }
    if (P->prec == TN_FP64) {
        // one plain-sampler launch per chain for the current state and one for
        // the proposal; the chain's sampler counts go to this context
        for (int m = 0; m < P->n; ++m)
            for (int j = 0; j < P->chains[m]; ++j) {
                const int g = P->first[m] + j;
                tn_ctx *k = P->kids[g];
                unsigned long long *own = k->counters;
                k->counters = ctx->counters;
                rc = tn_run_fp64(k, 1, 0, 0, 1, 0, P->os + (size_t)g * P->nso, true, P->slogq + g, P->sE + g);
                if (rc == TN_OK)
                    rc = tn_run_fp64(k, 1, seed, step, 1, (uint64_t)j, P->ps + (size_t)g * P->nso, false,
                                     P->plogq + g, P->pE + g);
                k->counters = own;
                if (rc) return tn_fail(ctx, rc, k->err);
            }
        if (!P->descs_ready && (rc = make_descs(ctx, P))) return rc;
    } else {
        if (!P->descs_ready && (rc = make_descs(ctx, P))) return rc;
        // one proposal per chain: the one-set-per-wave variant, whose second
        // team of a chain has no proposal and leaves at once
        const int NT = ((P->D + 15) / 16);
        const bool bf = P->prec == TN_BF16;
        const int v = NT <= 2 ? 1 : 0;
        if ((rc = tn_run_mfma_multi(ctx, NT, bf, v, P->sd_eval, T, 8 * T, P->Lxo, 0, 0, true))) return rc;
        if ((rc = tn_run_mfma_multi(ctx, NT, bf, v, P->sd_samp, T, 8 * T, P->Lxo, seed, step, false))) return rc;
    }
    if ((rc = tn_launch_accept_multi(ctx, P->ad, P->nacc, T, seed, step))) return rc;
    hipLaunchKernelGGL(k_uncut, dim3(T), dim3(PT_THREADS), (size_t)P->Lx * P->Ly, ctx->stream, P->pd, P->inst_of,
                       P->Lx, P->Ly, P->wx, P->wy, P->Lxo, P->Lyo, cr, cc, P->os, spins, energy, P->acc, accepted);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}

int tn_periodic_sweeps(tn_ctx *ctx, int nsweeps, uint64_t seed, uint64_t step, int8_t *spins, double *energy) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_periodic(ctx))) return rc;
    tn_periodic *P = per_of(ctx);
    if (!spins || !energy) return tn_fail(ctx, TN_EINVAL, "NULL buffer");
    if (nsweeps < 0 || nsweeps >= (1 << 18)) return tn_fail(ctx, TN_EINVAL, "nsweeps must be in 0..2^18-1");
    if ((P->wx && (P->Lx & 1)) || (P->wy && (P->Ly & 1)))
        return tn_fail(ctx, TN_EINVAL, "checkerboard sweeps need an even length along a wrapped direction");
    if (nsweeps > 0) {
        hipLaunchKernelGGL(k_per_metropolis, dim3(P->total), dim3(PT_THREADS), (size_t)P->Lx * P->Ly, ctx->stream,
                           P->pd, P->inst_of, P->Lx, P->Ly, P->wx, P->wy, nsweeps, spins, (uint32_t)seed,
                           (uint32_t)(seed >> 32), (uint32_t)step, ctx->counters);
        TN_HIP(ctx, hipGetLastError());
    }
    return tn_periodic_energy(ctx, spins, energy);
}

int tn_periodic_energy(tn_ctx *ctx, const int8_t *spins, double *energy) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_periodic(ctx))) return rc;
    tn_periodic *P = per_of(ctx);
    if (!spins || !energy) return tn_fail(ctx, TN_EINVAL, "NULL buffer");
    hipLaunchKernelGGL(k_uncut, dim3(P->total), dim3(PT_THREADS), (size_t)P->Lx * P->Ly, ctx->stream, P->pd,
                       P->inst_of, P->Lx, P->Ly, P->wx, P->wy, P->Lxo, P->Lyo, 0, 0, nullptr,
                       const_cast<int8_t *>(spins), energy, nullptr, nullptr);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}

int tn_periodic_link_overlap(tn_ctx *ctx, int n, const int8_t *a, const int8_t *b, int32_t *q) {
    (void)hipGetLastError();
    int rc;
    if ((rc = need_periodic(ctx))) return rc;
    tn_periodic *P = per_of(ctx);
    if (n < 0) return tn_fail(ctx, TN_EINVAL, "n < 0");
    if (n == 0) return TN_OK;
    if (!a || !b || !q) return tn_fail(ctx, TN_EINVAL, "NULL buffer");
    return tn_launch_link_overlap_lattice(ctx, P->Lx, P->Ly, P->wx, P->wy, n, a, b, q);
}

}  // extern "C"
