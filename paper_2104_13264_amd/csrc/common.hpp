// Shared definitions of the gfx950 TNMH library: the context, error handling,
// device helpers (Philox4x32-10, bond-leg factors, wavefront reductions).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/tnmh.h"

#define TN_MAX_D 64
#define TN_MDESC_SETS 8

// Device counters (uint64) kept per context.
enum {
    CNT_CLAMPS = 0,
    CNT_BOTH = 1,
    CNT_NEAR = 2,
    CNT_ACCEPTED = 3,
    CNT_PROPOSED = 4,
    CNT_DEGEN = 5,
    CNT_NOCONV = 6,
    CNT_FLIPS = 7,   // accepted single-spin flips of the Metropolis sweeps
    CNT_N = 8
};

// Launch shape chosen by tn_autotune for one instance (lattice, padded bond
// dimension and precision): the batched sampler's variant and the proposals
// per sampler launch in tn_mh_run.
struct tn_tuned {
    bool valid = false;
    int Lx = 0, Ly = 0, Dp = 0, prec = -1;
    int variant = 0;
    long proposals = 0;
};

struct tn_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;

    // instance
    int Lx = 0, Ly = 0, D = 0, Dp = 0, prec = TN_FP64, inst = 0;
    double beta = 0.0;
    bool has_env = false;
    bool has_ops64 = false, has_ops32 = false, has_ops16 = false;
    double logZ = 0.0;
    double env_build_ms = 0.0;

    // owned device copies of the couplings (fp64)
    double *Jh = nullptr, *Jv = nullptr, *h = nullptr;

    // environment stack: env[k][c][D][2][D], k = 0..Ly (k = 0 unused, k = Ly
    // trivial), bond dims dims[k][0..Lx], log-normalisers ell[k]
    double *env = nullptr;
    int *dims = nullptr;
    double *ell = nullptr;
    int *cst = nullptr;       // leftmost truncated column of env k, -1 if none
    bool has_cst = false;     // cst valid (environment built here, not installed)
    size_t env_cap = 0;       // elements allocated for env

    // sampler operands, one per row r = 0..Ly-1 and column:
    //   G64r[r][c][s][a][b]  = G_c(s)[a][b]  (row-major, fp64)
    //   G64c[r][c][s][b][a]  = G_c(s)[a][b]  (column-major, fp64)
    //   G32R / G32L          MFMA A-operand tiles of G and G^T (fp32)
    //   G16R / G16L          the same in bf16
    //   G64MR / G64ML        the same in fp64 (the batched fp64 path)
    double *G64r = nullptr, *G64c = nullptr;
    float *G32R = nullptr, *G32L = nullptr;
    uint16_t *G16R = nullptr, *G16L = nullptr;
    double *G64MR = nullptr, *G64ML = nullptr;
    size_t ops_cap64 = 0, ops_cap32 = 0, ops_cap16 = 0, ops_cap64m = 0;

    // Boltzmann factors per site: exp(+-beta h), exp(+-beta Jv above),
    // exp(+-beta Jh left), [Ly][Lx][6] fp64
    double *fac = nullptr;
    size_t fac_cap = 0;

    // compression: 0 successive SVD; n > 0 followed by n two-site variational
    // sweeps (tn_set_compression), with their scratch
    int fit_sweeps = 0;
    double *fbuf = nullptr;
    size_t fbuf_cap = 0;

    // environment-build scratch
    double *xbox = nullptr;   // [Lx][2D][2][2D]
    double *wbuf = nullptr;   // global work buffers when LDS is too small
    double *scal = nullptr;   // small device scalars (top overlap result ...)
    uint64_t *dstep = nullptr;  // device step base added to every MH step (graph replays)
    void *noalloc_scr = nullptr; // this device's fixed scratch of tn_sample_noalloc (not owned)
    const tn_ctx *proj_src = nullptr; // frozen evaluation: the build whose projectors it applies
    double *pscr = nullptr;     // its projection scratch (8 D^2 doubles)
    size_t pscr_cap = 0;
    std::vector<tn_ctx *> fkids;     // contexts of tn_logz_frozen's evaluations
    int noalloc_err = 0;         // hipError_t of its address lookup
    bool own_dstep = true;      // false for the instances of a batched context

    // batched uneven instances (tn_build_env_multi): one child context each
    std::vector<tn_ctx *> kids;
    std::vector<int> kid_chains;
    // device descriptor tables of tn_mh_step_multi, one per distinct set of
    // state buffers seen (at most TN_MDESC_SETS), with their host contents
    std::vector<void *> mdesc;
    std::vector<std::vector<unsigned char>> mdesc_host;
    bool has_multi = false;
    // incremental environment build (tn_build_env_begin .. _end)
    bool building = false;
    int build_step = 0;
    void *build_plan = nullptr;   // tn_build_plan, owned
    // two-sided derivative: the environments of the upside-down lattice,
    // built on demand and kept while the instance (env_gen) is unchanged
    tn_ctx *flip = nullptr;       // owned
    uint64_t env_gen = 0, flip_gen = ~0ull;
    // graph capture (tn_graph_begin .. tn_graph_end_and_replay)
    bool capturing = false;
    int graph_steps = 0;
    void *descs = nullptr;    // device descriptors of batched launches
    size_t descs_cap = 0;
    int *xdims = nullptr;     // [2][Lx+1]
    size_t xbox_cap = 0, wbuf_cap = 0;

    // sampler scratch (per-proposal right environments)
    void *gscr = nullptr;
    size_t gscr_cap = 0;

    // proposal buffers of tn_mh_step
    int8_t *pspins = nullptr;
    double *plogq = nullptr, *pE = nullptr;
    size_t pcap = 0;

    unsigned long long *counters = nullptr;   // CNT_N

    // adjoint scratch
    void *gradscr = nullptr;
    size_t gradscr_cap = 0;

    // autotuned launch shapes: this instance's, and per (bf16, bond class)
    // group of tn_mh_step_multi (-1: not tuned, variant 0)
    tn_tuned tuned;
    int multi_variant[2][5] = {{-1, -1, -1, -1, -1}, {-1, -1, -1, -1, -1}};

    // periodic lattices (tn_periodic_setup): tn_periodic, owned
    void *per = nullptr;

    // q-state Potts models (tn_potts_build_env, potts.hip): qd = d > 0 marks
    // a Potts context (env boxes D x d x D, h [Ly][Lx][d]); its factor
    // tables, sampler operands (both layouts) and build work area
    int qd = 0;
    double *pq = nullptr, *pG = nullptr, *pw = nullptr;
    size_t pq_cap = 0, pG_cap = 0, pw_cap = 0;
};

int tn_fail(tn_ctx *ctx, int code, const std::string &msg);
// Frees every buffer a context owns (not the context itself).
void tn_free_ctx(tn_ctx *ctx);
// Frees the periodic-lattice state of a context (periodic.hip).
void tn_periodic_free(tn_ctx *ctx);

#define TN_HIP(ctx, call)                                                          \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            return tn_fail((ctx), TN_EHIP, std::string(#call) + ": " +             \
                                               hipGetErrorString(e_));             \
    } while (0)

// grow a device buffer to at least `bytes`
int tn_ensure(tn_ctx *ctx, void **ptr, size_t *cap, size_t bytes);

// environment build (env_build.hip)
// One instance's environment build as the row kernels see it (device copy).
struct tn_env_desc {
    int Lx, Ly, D, fit;   // fit: two-site variational sweeps after the SVD sweep
    double beta;
    const double *Jh, *Jv, *h;
    double *env;
    int *dims;
    double *ell;
    int *cst;
    double *xbox;
    int *xdims;
    double *wbuf;
    double *scal;
    unsigned long long *counters;
    double *fbuf;         // the variational sweeps' scratch (fit > 0)
    // frozen contraction (tn_logz_frozen): after the MPO-MPS product of row
    // k, project onto the span the build of penv kept at its leftmost
    // truncated column pcst[k] (nothing where pcst[k] < 0); pscr: 8 D^2
    // doubles of scratch.  penv == nullptr: an ordinary build.
    const double *penv;
    const int *pdims;
    const int *pcst;
    double *pscr;
};
// Builds the environments of n instances together (one workgroup per
// instance and row step); fills each ctx's logZ.  ctxs[i] must have its
// instance set (couplings on the device).
int tn_env_build_many(tn_ctx *const *ctxs, int n, hipStream_t stream, std::string *err);
// The same in three parts (row steps s0..s1-1 per call, synchronised), for a
// build reported row chunk by row chunk.
struct tn_build_plan {
    int n = 0, maxLy = 0;
    // the three kernel classes: D <= 16 (256 threads), D 17-32 (512 threads),
    // both with their matrices in LDS, and D 33-64 (1024 threads); LDS bytes
    // 0 where no instance is of the class
    size_t lds_tiny = 0, lds_small = 0, lds_big = 0;
    // the variational sweeps' kernel (0: no instance fits)
    size_t lds_fit = 0;
    tn_env_desc *dd = nullptr;
    double ms = 0.0;
};
// threads of the row kernel that builds an instance of bond dimension D
__host__ __device__ constexpr int tn_env_class_threads(int D) { return D <= 16 ? 256 : (D <= 32 ? 512 : 1024); }
int tn_env_build_prepare(tn_ctx *const *ctxs, int n, hipStream_t stream, std::string *err,
                         tn_build_plan *plan);
int tn_env_build_steps(tn_build_plan *plan, int s0, int s1, hipStream_t stream, std::string *err);
int tn_env_build_finish(tn_ctx *const *ctxs, int n, tn_build_plan *plan, hipStream_t stream,
                        std::string *err);
// The top overlap of every instance of a plan after its row steps, and each
// instance's outcome in status[i] (device, int [n]): 0 usable, 1 Z~ not
// positive or not finite, 2 SVD not converged.  No synchronisation.
int tn_env_build_top_status(const tn_build_plan *plan, int *status, hipStream_t stream);
int tn_env_build_device(tn_ctx *ctx, double *logZ_out);
int tn_make_operands(tn_ctx *ctx, int prec);
// One instance's operand build as the batched kernels see it (the buffers
// of the instance's precision; the others NULL).
struct tn_ops_desc {
    int Lx, Ly, D, Dp;
    double beta;
    const double *Jh, *Jv, *h, *env;
    const int *dims;
    double *fac, *G64r, *G64c;
    float *G32R, *G32L;
    uint16_t *G16R, *G16L;
    double *G64MR, *G64ML;
};
// after tn_make_operands has allocated the context's operand buffers
tn_ops_desc tn_ops_desc_of(const tn_ctx *ctx, int prec);
// The operands of n instances (device descriptors) in two launches on
// ctx's stream; maxDp: the largest padded bond dimension among them.
int tn_make_operands_many(tn_ctx *ctx, const tn_ops_desc *descs, int n, int maxLx, int maxLy, int maxDp);

// samplers
// One instance's batched-sampler launch as the kernel sees it.  Block blk of
// the instance draws proposals 16 blk .. 16 blk + 15; blk0 is the first block
// of the instance in a launch over several instances.
struct tn_samp_desc {
    int B, Lx, Ly, per_step;
    const double *Jh, *Jv, *h, *fac;
    const void *GR, *GL;
    int8_t *S;
    double *logq, *energy;
    float *gscr;
    uint64_t first_id;
    uint32_t inst;
    int blk0;
    unsigned long long *counters;
};
inline tn_samp_desc tn_samp_desc_of(tn_ctx *ctx, int B, int8_t *S, double *logq, double *energy,
                                    float *gscr, int per_step, uint64_t first_id) {
    tn_samp_desc A;
    A.B = B;
    A.Lx = ctx->Lx;
    A.Ly = ctx->Ly;
    A.per_step = per_step;
    A.Jh = ctx->Jh;
    A.Jv = ctx->Jv;
    A.h = ctx->h;
    A.fac = ctx->fac;
    const bool bf16 = ctx->prec == TN_BF16;
    const bool f64 = ctx->prec == TN_FP64_MFMA;
    A.GR = bf16 ? (const void *)ctx->G16R : (f64 ? (const void *)ctx->G64MR : (const void *)ctx->G32R);
    A.GL = bf16 ? (const void *)ctx->G16L : (f64 ? (const void *)ctx->G64ML : (const void *)ctx->G32L);
    A.S = S;
    A.logq = logq;
    A.energy = energy;
    A.gscr = gscr;
    A.first_id = first_id;
    A.inst = (uint32_t)ctx->inst;
    A.blk0 = 0;
    A.counters = ctx->counters;
    return A;
}
// Scratch bytes of the batched sampler for `batch` proposals: both spins' y
// tiles (fp32, 16 proposals x Dp) of every column, per 16-proposal unit, for
// whole teams (up to eight units).
inline size_t tn_mfma_scratch_bytes(const tn_ctx *ctx, int batch) {
    const int units = ((batch + 127) / 128) * 8;
    const size_t elem = ctx->prec == TN_FP64_MFMA ? sizeof(double) : sizeof(float);
    return (size_t)units * ctx->Lx * 2 * (size_t)ctx->Dp * 16 * elem;
}
// Scratch bytes of the plain fp64 sampler: per proposal both spins' right
// environments of every column of the row in flight.
inline size_t tn_fp64_scratch_bytes(const tn_ctx *ctx, int batch) {
    return (size_t)batch * ctx->Lx * 2 * ctx->D * sizeof(double);
}
// Launch variants of the batched sampler for bond class NT = Dp / 16 and its
// operands (same arithmetic, different launch shape; sampler_mfma.hip): four
// for D <= 32, two for BF16 D 33-64, one for FP32 D 33-64 (no recomputing
// variant there: it would need every one of a lane's 512 registers).
constexpr int tn_team_variants(int NT, bool bf16) { return NT <= 2 ? 4 : (bf16 ? 2 : 1); }
// Whether tn_autotune's choice applies to the context's current instance
// (same lattice, padded bond dimension and precision), and its variant (0 if
// there is none).
inline bool tn_tuned_here(const tn_ctx *ctx) {
    const tn_tuned &t = ctx->tuned;
    return t.valid && t.Lx == ctx->Lx && t.Ly == ctx->Ly && t.Dp == ctx->Dp && t.prec == ctx->prec;
}
inline int tn_ctx_variant(const tn_ctx *ctx) { return tn_tuned_here(ctx) ? ctx->tuned.variant : 0; }
// eval: the descriptors' spins are given and only ln q and E are computed
int tn_run_mfma_multi(tn_ctx *ctx, int NT, bool bf16, int variant, const tn_samp_desc *descs, int n,
                      int blocks, int maxLx, uint64_t seed, uint64_t step0, bool eval = false);
// tn_mh_step_multi's proposal draws: every instance's proposal buffers and
// scratch (allocated on first use; refused while capturing), and the sampler
// descriptors grouped by (bf16, bond class), each group one launch.
struct tn_multi_group {
    int NT;
    bool bf16;
    int first, count, blocks, maxLx;
};
int tn_multi_prepare(tn_ctx *ctx);
void tn_multi_groups(tn_ctx *ctx, std::vector<tn_samp_desc> &sd, std::vector<tn_multi_group> &groups);

// Samplers: proposal j of a launch has id first_id + j % per_step and MH step
// step0 + j / per_step.
// scr: the sampler's scratch (at least tn_fp64_scratch_bytes or
// tn_mfma_scratch_bytes), or nullptr for the context's own buffer, allocated
// or grown as needed.
int tn_run_fp64(tn_ctx *ctx, int batch, uint64_t seed, uint64_t step0, int per_step,
                uint64_t first_id, int8_t *spins, bool eval, double *logq,
                double *energy, void *scr = nullptr);
// variant: launch variant of the batched sampler, -1 for the context's
int tn_run_mfma(tn_ctx *ctx, int batch, uint64_t seed, uint64_t step0, int per_step,
                uint64_t first_id, int8_t *spins, bool eval, double *logq,
                double *energy, int variant = -1, void *scr = nullptr);

// q-state Potts sampler (potts.hip): the plain fp64 draw with d-way
// conditionals; scr as for tn_run_fp64 (tn_potts_scratch_bytes)
int tn_run_potts(tn_ctx *ctx, int batch, uint64_t seed, uint64_t step0, int per_step,
                 uint64_t first_id, int8_t *states, bool eval, double *logq, double *energy,
                 void *scr = nullptr);
inline size_t tn_potts_scratch_bytes(const tn_ctx *ctx, int batch) {
    return (size_t)batch * ctx->Lx * ctx->qd * ctx->D * sizeof(double);
}

// Metropolis sweeps of `chains` states in place (metropolis.hip)
int tn_launch_metropolis(tn_ctx *ctx, int chains, int nsweeps, uint64_t seed, uint64_t step, int8_t *spins);

// Link overlaps of configuration pairs (stats.hip)
int tn_launch_link_overlap(tn_ctx *ctx, int n, const int8_t *a, const int8_t *b, int32_t *q);
// The same on a given lattice, with the bonds that wrap along x / y if wx / wy
int tn_launch_link_overlap_lattice(tn_ctx *ctx, int Lx, int Ly, int wx, int wy, int n, const int8_t *a,
                                   const int8_t *b, int32_t *q);

// MH accept kernel launcher (mh.hip)
// One instance's MH acceptance launch as the kernel sees it.
struct tn_acc_desc {
    int chains, nsite;
    double beta;
    uint32_t inst;
    int blk0;
    const int8_t *pspins;
    const double *plogq, *pE;
    int8_t *sspins;
    double *slogq, *sE;
    uint8_t *accepted;
    unsigned long long *counters;
    double *eser;   // state energy after the step, [chains], or NULL
};
int tn_launch_accept_multi(tn_ctx *ctx, const tn_acc_desc *descs, int n, int total_chains,
                           uint64_t seed, uint64_t step);
int tn_launch_accept(tn_ctx *ctx, int chains, uint64_t seed, uint64_t step,
                     const int8_t *prop_spins, const double *prop_logq,
                     const double *prop_energy, int8_t *state_spins, double *state_logq,
                     double *state_energy, uint8_t *accepted,
                     double *energy_series = nullptr);

// adjoint (grad.hip)
// upper == nullptr: the frozen-truncation derivative of ln Z~; otherwise the
// two-sided estimate with `upper` holding the upside-down lattice's envs.
int tn_grad_device(tn_ctx *ctx, const tn_ctx *upper, double *dJh, double *dJv, double *dbeta);

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// 4x32 S-box with two 32x32->64 multiplies, Weyl-incremented key.  Each
// product is taken whole (one v_mad_u64_u32 instead of separate low and high
// multiplies, both quarter rate).
__device__ __forceinline__ uint4 tn_philox(uint4 ctr, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        if (rnd) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * ctr.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * ctr.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        ctr = make_uint4(hi1 ^ ctr.y ^ k0, lo1, hi0 ^ ctr.w ^ k1, lo0);
    }
    return ctr;
}

__device__ __forceinline__ double tn_u01(uint32_t x) {
    return ((double)x + 0.5) * 2.3283064365386963e-10;   // 2^-32
}

__device__ __forceinline__ uint32_t tn_word(uint4 v, int w) {
    return w == 0 ? v.x : (w == 1 ? v.y : (w == 2 ? v.z : v.w));
}

// Bond-leg factors of W(s,s') = exp(K s s') = P Q (App. A):
//   P(s,0) = sqrt(cosh K), P(s,1) = s sqrt|sinh K|
//   Q(0,s) = sqrt(cosh K), Q(1,s) = sign(K) s sqrt|sinh K|
// spin index 0 is s = +1, index 1 is s = -1.
__device__ __forceinline__ double tn_pleg(double K, int sidx, int mu) {
    const double s = sidx ? -1.0 : 1.0;
    return mu == 0 ? sqrt(cosh(K)) : s * sqrt(fabs(sinh(K)));
}
__device__ __forceinline__ double tn_qleg(double K, int mu, int sidx) {
    const double s = sidx ? -1.0 : 1.0;
    const double sg = K >= 0.0 ? 1.0 : -1.0;
    return mu == 0 ? sqrt(cosh(K)) : sg * s * sqrt(fabs(sinh(K)));
}

// Wavefront reductions on the VALU: quad permutations, the half-row and row
// mirrors (DPP) and the 16- and 32-lane swaps of gfx950, no LDS round trips.
// Every lane ends with the same value, combined in the same order.
namespace tn_detail {
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}
struct Pair32 {
    uint32_t a, b;
};
// the partner's value in each of the six combining steps
template <int STEP>
__device__ __forceinline__ uint32_t partner32(uint32_t v) {
    if constexpr (STEP == 0) return dpp32<0xB1>(v);          // quad_perm [1,0,3,2]
    else if constexpr (STEP == 1) return dpp32<0x4E>(v);     // quad_perm [2,3,0,1]
    else if constexpr (STEP == 2) return dpp32<0x141>(v);    // row_half_mirror
    else if constexpr (STEP == 3) return dpp32<0x140>(v);    // row_mirror
    else if constexpr (STEP == 4) {
        auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (threadIdx.x & 16) ? r[0] : r[1];
    } else {
        auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (threadIdx.x & 32) ? r[0] : r[1];
    }
}
template <int STEP>
__device__ __forceinline__ float partner(float v) {
    return __uint_as_float(partner32<STEP>(__float_as_uint(v)));
}
template <int STEP>
__device__ __forceinline__ double partner(double v) {
    const uint32_t lo = partner32<STEP>((uint32_t)__double2loint(v));
    const uint32_t hi = partner32<STEP>((uint32_t)__double2hiint(v));
    return __hiloint2double((int)hi, (int)lo);
}
template <int STEP>
__device__ __forceinline__ int partner(int v) {
    return (int)partner32<STEP>((uint32_t)v);
}
}  // namespace tn_detail

template <typename T>
__device__ __forceinline__ T tn_wave_sum(T v) {
    using namespace tn_detail;
    v = v + partner<0>(v);
    v = v + partner<1>(v);
    v = v + partner<2>(v);
    v = v + partner<3>(v);
    v = v + partner<4>(v);
    v = v + partner<5>(v);
    return v;
}
template <typename T>
__device__ __forceinline__ T tn_wave_max(T v) {
    using namespace tn_detail;
    v = fmax(v, partner<0>(v));
    v = fmax(v, partner<1>(v));
    v = fmax(v, partner<2>(v));
    v = fmax(v, partner<3>(v));
    v = fmax(v, partner<4>(v));
    v = fmax(v, partner<5>(v));
    return v;
}

// Sum over the 16 lanes of a row (lanes 16r .. 16r+15): quad permutations
// and the half-row and row mirrors; every lane of the row ends with the same
// value.
template <typename T>
__device__ __forceinline__ T tn_row16_sum(T v) {
    using namespace tn_detail;
    v = v + partner<0>(v);
    v = v + partner<1>(v);
    v = v + partner<2>(v);
    v = v + partner<3>(v);
    return v;
}

// block-wide sum over all threads; every thread receives the total.
// `red` must hold blockDim.x/64 doubles of LDS.
__device__ __forceinline__ double tn_block_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    v = tn_wave_sum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}
__device__ __forceinline__ double tn_block_max(double v, double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    v = tn_wave_max(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t = fmax(t, red[i]);
    return t;
}
