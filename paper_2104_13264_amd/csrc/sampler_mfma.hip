// Batched sampler on the matrix cores: the same sequential draw and the same
// conditionals as the plain path (Sec. 2 Eqs. bayes, pi-approx; App. A
// Eq. proba-ratio-apx), with the per-column products run as 16x16 MFMA tiles.
//
// A workgroup owns 16 proposals (the N dimension of every tile) for the whole
// lattice; its 2*NT waves (Dp = 16*NT padded bond) each own one output tile
// (spin s, 16-row block mo) of every column product, so the 16 proposals'
// work is spread over 2*NT SIMDs.  Per column:
//   right sweep  y_s[mo] = G_c(s)[mo,:] r_s      (NQ chained MFMAs, K = Dp)
//                tiles exchanged through LDS (double buffered, one barrier),
//                r_s' = sum_s W(s',s) v_c(s) y_s rescaled by a common 2^-e,
//                every wave rebuilding its own next B operand r_{s_w}
//   left sweep   w(s) = v hf <Lam, y_s>   (y_s re-read from this
//                workgroup's scratch), p+ and the draw in fp64 on every wave
//                (bitwise identical), Lam_s'[mo] = G_c(s)^T[mo,:] Lam,
//                exchanged and selected by the drawn spin.
// The accumulator layout of tile mt (lane l, register i -> row 4(l/16)+i,
// column l%16) is exactly the B-operand layout of k-chunk q = 4 mt + i of the
// next product, so the recurrences stay in registers; the A operands (the
// shared environment) are pre-permuted to match (operands.hip).
//
// ln q is accumulated as a product of the drawn probabilities in fp64 with a
// separate binary exponent, and evaluated once at the end.
#include "common.hpp"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

#define TN_MAX_LX 256

__device__ __forceinline__ int pow2_exponent_f(float m) {
    int e = 0;
    if (m > 0.0f && m <= 3.0e38f) frexpf(m, &e);
    return e;
}

__device__ __forceinline__ short bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// A operand of one output tile for one column: the NQ = 4 NT k-chunks of the
// fp32 16x16x4 product, or the NT chunks of the bf16 16x16x16 product.
template <int NT, bool BF16>
struct ATile;

template <int NT>
struct ATile<NT, false> {
    static constexpr int NQ = 4 * NT;
    float a[NQ];
    __device__ __forceinline__ void load(const void *base, int lane) {
        const float *A = (const float *)base;
#pragma unroll
        for (int q = 0; q < NQ; ++q) a[q] = A[q * 64 + lane];
    }
    __device__ __forceinline__ floatx4 mul(const floatx4 (&x)[NT]) const {
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], x[q >> 2][q & 3], acc, 0, 0, 0);
        return acc;
    }
};

template <int NT>
struct ATile<NT, true> {
    shortx4 a[NT];
    __device__ __forceinline__ void load(const void *base, int lane) {
        const shortx4 *A = (const shortx4 *)base;
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) a[mt] = A[mt * 64 + lane];
    }
    __device__ __forceinline__ floatx4 mul(const floatx4 (&x)[NT]) const {
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
            shortx4 bv;
            bv[0] = bf16_rne(x[mt][0]);
            bv[1] = bf16_rne(x[mt][1]);
            bv[2] = bf16_rne(x[mt][2]);
            bv[3] = bf16_rne(x[mt][3]);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mt], bv, acc, 0, 0, 0);
        }
        return acc;
    }
};

template <int NT, bool BF16>
__device__ __forceinline__ const void *tile_ptr(const void *G, size_t site, int sw, int mow) {
    constexpr int Dp = 16 * NT;
    constexpr size_t TILE = BF16 ? (size_t)NT * 64 * 4 : (size_t)4 * NT * 64;   // elements
    const size_t off = site * 2 * Dp * Dp + ((size_t)sw * NT + mow) * TILE;
    return BF16 ? (const void *)((const uint16_t *)G + off) : (const void *)((const float *)G + off);
}

// Columns of the environment tiles (and, for the drawing group, of the stored
// y_s tiles) are kept in a ring of PF registers sets: the set used at column
// step t is refilled with step t + PF.  The step loop is unrolled by PF so that
// the ring is indexed statically and no register copy waits for a load.
template <int NT, bool BF16>
constexpr int prefetch_depth() { return (NT <= 2 || BF16) ? 3 : 2; }

// Sum (or max) over the four 16-lane rows of a wavefront, the same result in
// every lane: the 32-lane and 16-lane swaps of gfx950 (VALU, no LDS traffic).
__device__ __forceinline__ float rows4_sum(float v) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}
__device__ __forceinline__ float rows4_max(float v) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
    auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return fmaxf(__uint_as_float(q[0]), __uint_as_float(q[1]));
}

// Snake order: row r is drawn left to right when r is even, right to left
// when odd.  Before a row is drawn, the environments of its free columns are
// swept from its far end; that sweep runs in the same column order as the
// drawing of the row above, so the two run side by side: phase p pairs the
// environment sweep of row p (group p & 1) with the drawing of row p-1 (the
// other group), one column per step and one barrier per step, and the drawn
// spin of a column is in LDS before the environment sweep of the row below
// needs it.  A rightward phase multiplies by G^T (GL tiles), a leftward one by
// G (GR tiles), for both groups.
//
// LDS arrays indexed by proposal keep the proposal index innermost, so the 16
// proposals of a wavefront touch 16 consecutive entries (no bank conflicts).
template <int NT, bool BF16>
__global__ void __launch_bounds__(256 * NT)
k_sampler_mfma(int B, int Lx, int Ly, const double *__restrict__ Jh,
               const double *__restrict__ Jv, const double *__restrict__ h,
               const double *__restrict__ fac, const void *__restrict__ GRv,
               const void *__restrict__ GLv, int8_t *__restrict__ S, int eval,
               double *__restrict__ logq, double *__restrict__ energy,
               float *__restrict__ gscr, uint32_t k0, uint32_t k1, uint64_t first_id,
               uint32_t step, uint32_t inst, unsigned long long *__restrict__ counters) {
    constexpr int NW = 2 * NT;                        // waves per group
    constexpr int PF = prefetch_depth<NT, BF16>();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gp = w / NW, wl = w % NW;
    const int sw = wl / NT, mow = wl % NT;
    const int n = lane & 15, grp = lane >> 4;
    const int b = blockIdx.x * 16 + n;
    const bool valid = b < B;
    const bool leader = (wl == 0 && grp == 0);        // one lane per proposal per group

    __shared__ floatx4 xch[2][2][2][NT][64];         // [group][buf][s][mo][lane]
    __shared__ int8_t rows[2][TN_MAX_LX][16];         // spins by row parity
    __shared__ uint32_t uni[TN_MAX_LX][16];           // random words of the drawn row
    __shared__ float mixP[TN_MAX_LX][2][2][2];        // [c][s_up][s_w][s]
    __shared__ double vS[TN_MAX_LX][2][2][2];         // [c][s_up][s_prev][s]
    __shared__ double lqx[2][16][2];                  // ln q parts per group

    const size_t gstride = (size_t)2 * NT * 64 * 4;   // floats per column
    float *gwg = gscr + (size_t)(blockIdx.x * 2 + gp) * Lx * gstride;
    const int NTH = blockDim.x;

    double mant = 1.0, E = 0.0;
    int mexp = 0;
    unsigned long long n_clamp = 0, n_both = 0, n_near = 0;
    int buf = 0;

    for (int p = 0; p <= Ly; ++p) {
        const bool hasP = p < Ly, hasS = p >= 1;
        const bool isP = hasP && gp == (p & 1);
        const bool isS = hasS && gp != (p & 1);
        const bool rightward = (p & 1) != 0;          // column order of this phase
        const int rS = p - 1;                          // row drawn in this phase
        // ---- phase set-up: factor tables, random words, given spins
        for (int t = threadIdx.x; t < Lx * 8; t += NTH) {
            const int c = t >> 3, su = (t >> 2) & 1, x = (t >> 1) & 1, s = t & 1;
            if (hasP) {   // environment sweep of row p: W(s_w = x, s) v_c(s; s_up)
                const double *f = fac + ((size_t)p * Lx + c) * 6;
                const int cb = rightward ? c + 1 : c;   // bond towards the next column
                double Wv = 1.0;
                if (cb >= 1 && cb <= Lx - 1) Wv = fac[((size_t)p * Lx + cb) * 6 + ((x == s) ? 4 : 5)];
                const double v = f[s] * f[2 + (su ^ s)];
                mixP[c][su][x][s] = (float)(Wv * v);
            }
            if (hasS) {   // drawing of row p-1: v_c(s; s_up) hf(s; s_prev)
                const double *f = fac + ((size_t)rS * Lx + c) * 6;
                const int cb = rightward ? c : c + 1;   // bond to the previous column
                double hf = 1.0;
                if (cb >= 1 && cb <= Lx - 1) hf = fac[((size_t)rS * Lx + cb) * 6 + ((x == s) ? 4 : 5)];
                vS[c][su][x][s] = f[s] * f[2 + (su ^ s)] * hf;
            }
        }
        if (hasS && !eval) {   // random words of row p-1
            for (int t = threadIdx.x; t < 16 * Lx; t += NTH) {
                const int c = t >> 4, nn = t & 15;
                const int i = rS * Lx + c;
                const uint4 x = tn_philox(make_uint4((uint32_t)(i >> 2),
                                                     (uint32_t)(first_id + blockIdx.x * 16 + nn),
                                                     step, (inst << 2) | 0u), k0, k1);
                uni[c][nn] = tn_word(x, i & 3);
            }
        }
        if (hasS && eval) {   // the given spins of row p-1
            for (int t = threadIdx.x; t < 16 * Lx; t += NTH) {
                const int nn = t / Lx, c = t % Lx;
                const int bb = blockIdx.x * 16 + nn;
                rows[rS & 1][c][nn] = bb < B ? S[((size_t)bb * Ly + rS) * Lx + c] : (int8_t)1;
            }
        }
        __syncthreads();

        const size_t rowP = (size_t)p * Lx, rowSb = (size_t)rS * Lx;
        const void *Gph = rightward ? GLv : GRv;
        floatx4 vec[NT];   // r_{s_w} (environment sweep) or Lam (drawing)
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) vec[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        if (grp == 0) vec[0][0] = 1.0f;
        const size_t rbase = isP ? rowP : rowSb;
        auto colof = [&](int t) { return rightward ? t : Lx - 1 - t; };
        auto gptr = [&](int c, int s2, int mo) {
            return (const floatx4 *)(gwg + c * gstride + (((size_t)s2 * NT + mo) * 64 + lane) * 4);
        };
        ATile<NT, BF16> a[PF];
        floatx4 g[PF][2][NT];   // stored y_s tiles of the drawn row (drawing group)
        if (isP || isS) {
#pragma unroll
            for (int k = 0; k < PF; ++k)
                a[k].load(tile_ptr<NT, BF16>(Gph, rbase + colof(min(k, Lx - 1)), sw, mow), lane);
        }
        if (isS) {
#pragma unroll
            for (int k = 0; k < PF; ++k)
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
                    for (int mo = 0; mo < NT; ++mo) g[k][s2][mo] = *gptr(colof(min(k, Lx - 1)), s2, mo);
        }
        const int8_t(*prowP)[16] = rows[(p + 1) & 1];   // row p-1 (above row p)
        const int8_t(*prowS)[16] = rows[p & 1];         // row p-2 (above row p-1)
        int8_t(*crowS)[16] = rows[(p + 1) & 1];         // row p-1, written by the drawing

        // One loop per role over whole turns of the ring, then the remaining
        // steps; the loads are unconditional (the last columns re-read the final
        // one), so that the compiler can count the loads in flight and waits
        // only for the ring entry it uses.
        if (isS) {
            int sprev = 0;   // index of the previous spin (0: +1, 1: -1); unused at t = 0
            auto stepS = [&](int k, int t) {
                const int c = colof(t);
                const int cn = colof(min(t + PF, Lx - 1));
                // the product with G_c(s_w) does not depend on the draw: issue it first
                const floatx4 acc = a[k].mul(vec);
                float d0 = 0.0f, d1 = 0.0f;
#pragma unroll
                for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        d0 = fmaf(vec[mo][i], g[k][0][mo][i], d0);
                        d1 = fmaf(vec[mo][i], g[k][1][mo][i], d1);
                    }
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
                    for (int mo = 0; mo < NT; ++mo) g[k][s2][mo] = *gptr(cn, s2, mo);
                a[k].load(tile_ptr<NT, BF16>(Gph, rbase + cn, sw, mow), lane);
                d0 = rows4_sum(d0);
                d1 = rows4_sum(d1);
                const int su = rS > 0 ? (prowS[c][n] > 0 ? 0 : 1) : 0;
                double w0 = vS[c][su][sprev][0] * (double)d0;
                double w1 = vS[c][su][sprev][1] * (double)d1;
                n_clamp += (w0 < 0.0) + (w1 < 0.0);
                w0 = fmax(w0, 0.0);
                w1 = fmax(w1, 0.0);
                const double tot = w0 + w1;
                const bool bad = !(tot > 0.0 && tot <= 1.79e308);
                n_both += bad;
                const double pp = bad ? 0.5 : w0 / tot;
                int s;
                if (eval) {
                    s = crowS[c][n];
                } else {
                    const double u = tn_u01(uni[c][n]);
                    s = (u < pp) ? 1 : -1;
                    n_near += fabs(u - pp) < 1e-6;
                    if (leader) crowS[c][n] = (int8_t)s;
                }
                int e2;
                mant = frexp(mant * (s > 0 ? pp : 1.0 - pp), &e2);
                mexp += e2;
                sprev = s > 0 ? 0 : 1;
                xch[gp][buf][sw][mow][lane] = acc;
                __syncthreads();
                float mx = 0.0f;
#pragma unroll
                for (int mo = 0; mo < NT; ++mo) {
                    vec[mo] = s > 0 ? xch[gp][buf][0][mo][lane] : xch[gp][buf][1][mo][lane];
#pragma unroll
                    for (int i = 0; i < 4; ++i) mx = fmaxf(mx, fabsf(vec[mo][i]));
                }
                const int e = pow2_exponent_f(rows4_max(mx));
#pragma unroll
                for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                    for (int i = 0; i < 4; ++i) vec[mo][i] = ldexpf(vec[mo][i], -e);
                buf ^= 1;
            };
            int t0 = 0;
            for (; t0 + PF <= Lx; t0 += PF) {
#pragma unroll
                for (int k = 0; k < PF; ++k) stepS(k, t0 + k);
            }
#pragma unroll
            for (int k = 0; k < PF - 1; ++k)
                if (t0 + k < Lx) stepS(k, t0 + k);
        } else if (isP) {
            auto stepP = [&](int k, int t) {
                const int c = colof(t);
                const floatx4 acc = a[k].mul(vec);
                *(floatx4 *)gptr(c, sw, mow) = acc;
                a[k].load(tile_ptr<NT, BF16>(Gph, rbase + colof(min(t + PF, Lx - 1)), sw, mow), lane);
                xch[gp][buf][sw][mow][lane] = acc;
                __syncthreads();
                if (t + 1 < Lx) {
                    floatx4 y[2][NT];
                    float mx = 0.0f;
#pragma unroll
                    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
                        for (int mo = 0; mo < NT; ++mo) {
                            y[s2][mo] = xch[gp][buf][s2][mo][lane];
#pragma unroll
                            for (int i = 0; i < 4; ++i) mx = fmaxf(mx, fabsf(y[s2][mo][i]));
                        }
                    const int e = pow2_exponent_f(rows4_max(mx));
                    const int su = p > 0 ? (prowP[c][n] > 0 ? 0 : 1) : 0;
                    const float m0 = mixP[c][su][sw][0], m1 = mixP[c][su][sw][1];
#pragma unroll
                    for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            vec[mo][i] = ldexpf(m0 * y[0][mo][i] + m1 * y[1][mo][i], -e);
                }
                buf ^= 1;
            };
            int t0 = 0;
            for (; t0 + PF <= Lx; t0 += PF) {
#pragma unroll
                for (int k = 0; k < PF; ++k) stepP(k, t0 + k);
            }
#pragma unroll
            for (int k = 0; k < PF - 1; ++k)
                if (t0 + k < Lx) stepP(k, t0 + k);
        } else {   // idle group (first and last phase): keep the barrier count
            for (int t = 0; t < Lx; ++t) {
                __syncthreads();
                buf ^= 1;
            }
        }
        __syncthreads();   // the drawn row is complete in LDS

        if (hasS) {
            // energy of row p-1 (Eq. ising: field, bonds in the row, bonds to the row above)
            if (gp == 0 && leader) {
                const int8_t(*cur)[16] = rows[(p + 1) & 1];
                const int8_t(*abv)[16] = rows[p & 1];
                double e = 0.0;
                for (int c = 0; c < Lx; ++c) {
                    const int sc = cur[c][n];
                    if (h) e -= h[rowSb + c] * sc;
                    if (c > 0) e -= Jh[(size_t)rS * (Lx - 1) + c - 1] * (double)(cur[c - 1][n] * sc);
                    if (rS > 0) e -= Jv[(size_t)(rS - 1) * Lx + c] * (double)(abv[c][n] * sc);
                }
                E += e;
            }
            if (!eval) {
                for (int t = threadIdx.x; t < 16 * Lx; t += NTH) {
                    const int nn = t / Lx, c = t % Lx;
                    const int bb = blockIdx.x * 16 + nn;
                    if (bb < B) S[((size_t)bb * Ly + rS) * Lx + c] = rows[(p + 1) & 1][c][nn];
                }
            }
        }
    }
    // combine the two groups' ln q parts; flush the counters
    if (leader) {
        lqx[gp][n][0] = mant;
        lqx[gp][n][1] = (double)mexp;
        if (valid) {
            if (n_clamp) atomicAdd(&counters[CNT_CLAMPS], n_clamp);
            if (n_both) atomicAdd(&counters[CNT_BOTH], n_both);
            if (n_near && !eval) atomicAdd(&counters[CNT_NEAR], n_near);
        }
    }
    __syncthreads();
    if (gp == 0 && leader && valid) {
        logq[b] = (log(lqx[0][n][0]) + log(lqx[1][n][0])) +
                  (lqx[0][n][1] + lqx[1][n][1]) * 0.69314718055994530942;
        energy[b] = E;
    }
}

template <int NT, bool BF16>
int launch_mfma(tn_ctx *ctx, int B, int8_t *S, bool eval, double *logq, double *energy,
                float *g, uint64_t seed, uint64_t step, uint64_t first_id) {
    const int blocks = (B + 15) / 16;
    const void *GR = BF16 ? (const void *)ctx->G16R : (const void *)ctx->G32R;
    const void *GL = BF16 ? (const void *)ctx->G16L : (const void *)ctx->G32L;
    hipLaunchKernelGGL((k_sampler_mfma<NT, BF16>), dim3(blocks), dim3(256 * NT), 0, ctx->stream,
                       B, ctx->Lx, ctx->Ly, ctx->Jh, ctx->Jv, ctx->h, ctx->fac, GR, GL, S,
                       eval ? 1 : 0, logq, energy, g, (uint32_t)seed, (uint32_t)(seed >> 32),
                       first_id, (uint32_t)step, (uint32_t)ctx->inst, ctx->counters);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}

template <bool BF16>
int dispatch_nt(tn_ctx *ctx, int B, int8_t *S, bool eval, double *logq, double *energy,
                float *g, uint64_t seed, uint64_t step, uint64_t first_id) {
    switch (ctx->Dp / 16) {
    case 1: return launch_mfma<1, BF16>(ctx, B, S, eval, logq, energy, g, seed, step, first_id);
    case 2: return launch_mfma<2, BF16>(ctx, B, S, eval, logq, energy, g, seed, step, first_id);
    case 3: return launch_mfma<3, BF16>(ctx, B, S, eval, logq, energy, g, seed, step, first_id);
    case 4: return launch_mfma<4, BF16>(ctx, B, S, eval, logq, energy, g, seed, step, first_id);
    default: return tn_fail(ctx, TN_EINVAL, "bond dimension above 64");
    }
}

}  // namespace

int tn_run_mfma(tn_ctx *ctx, int batch, uint64_t seed, uint64_t step, uint64_t first_id,
                int8_t *spins, bool eval, double *logq, double *energy) {
    if (batch == 0) return TN_OK;
    if (ctx->Lx > TN_MAX_LX) return tn_fail(ctx, TN_EINVAL, "Lx above 256");
    const int blocks = (batch + 15) / 16;
    const size_t need = (size_t)blocks * 2 * ctx->Lx * 2 * (ctx->Dp / 16) * 64 * 4 * sizeof(float);
    int rc;
    if ((rc = tn_ensure(ctx, &ctx->gscr, &ctx->gscr_cap, need))) return rc;
    float *g = (float *)ctx->gscr;
    if (ctx->prec == TN_BF16)
        return dispatch_nt<true>(ctx, batch, spins, eval, logq, energy, g, seed, step, first_id);
    return dispatch_nt<false>(ctx, batch, spins, eval, logq, energy, g, seed, step, first_id);
}
