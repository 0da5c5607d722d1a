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

// Columns of the environment tiles are prefetched PF columns ahead (two for
// the fp32 tiles of the largest bonds, to stay within the register file).
template <int NT, bool BF16>
constexpr int prefetch_depth() { return (NT <= 2 || BF16) ? 3 : 2; }

template <int NT, bool BF16>
__global__ void __launch_bounds__(128 * NT)
k_sampler_mfma(int B, int Lx, int Ly, const double *__restrict__ Jh,
               const double *__restrict__ Jv, const double *__restrict__ h,
               const double *__restrict__ fac, const void *__restrict__ GRv,
               const void *__restrict__ GLv, int8_t *__restrict__ S, int eval,
               double *__restrict__ logq, double *__restrict__ energy,
               float *__restrict__ gscr, uint32_t k0, uint32_t k1, uint64_t first_id,
               uint32_t step, uint32_t inst, unsigned long long *__restrict__ counters) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int sw = w / NT, mow = w % NT;
    const int n = lane & 15, grp = lane >> 4;
    const int b = blockIdx.x * 16 + n;
    const bool valid = b < B;
    const bool leader = (w == 0 && grp == 0 && valid);

    __shared__ floatx4 xch[2][2][NT][64];
    __shared__ int8_t rows[2][16][TN_MAX_LX];
    __shared__ double sfac[TN_MAX_LX][6];   // Boltzmann factors of the current row
    __shared__ double scpl[TN_MAX_LX][3];   // h, Jh to the left, Jv to the row above

    float *gwg = gscr + (size_t)blockIdx.x * Lx * 2 * NT * 64 * 4;
    const size_t gstride = (size_t)2 * NT * 64 * 4;   // floats per column

    double mant = 1.0;
    int mexp = 0;
    double E = 0.0;
    int buf = 0;
    uint4 blk = make_uint4(0, 0, 0, 0);
    int blk_id = -1;

    for (int r = 0; r < Ly; ++r) {
        const int8_t *prow = rows[(r + 1) & 1][n];   // row r-1
        int8_t *crow = rows[r & 1][n];
        for (int t = threadIdx.x; t < Lx; t += blockDim.x) {
            const double *f = fac + ((size_t)r * Lx + t) * 6;
#pragma unroll
            for (int q = 0; q < 6; ++q) sfac[t][q] = f[q];
            scpl[t][0] = h ? h[(size_t)r * Lx + t] : 0.0;
            scpl[t][1] = t > 0 ? Jh[(size_t)r * (Lx - 1) + t - 1] : 0.0;
            scpl[t][2] = r > 0 ? Jv[(size_t)(r - 1) * Lx + t] : 0.0;
        }
        __syncthreads();

        // ---- right sweep: rv = r_{sw} over all Dp components
        floatx4 rv[NT];
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) rv[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        if (grp == 0) rv[0][0] = 1.0f;
        const size_t rbase = (size_t)r * Lx;
        constexpr int PF = prefetch_depth<NT, BF16>();
        ATile<NT, BF16> a0, a1, a2;
        a0.load(tile_ptr<NT, BF16>(GRv, rbase + Lx - 1, sw, mow), lane);
        a1.load(tile_ptr<NT, BF16>(GRv, rbase + max(Lx - 2, 0), sw, mow), lane);
        if constexpr (PF == 3) a2.load(tile_ptr<NT, BF16>(GRv, rbase + max(Lx - 3, 0), sw, mow), lane);
        for (int c = Lx - 1; c >= 0; --c) {
            const floatx4 acc = a0.mul(rv);
            a0 = a1;
            if constexpr (PF == 3) {
                a1 = a2;
                a2.load(tile_ptr<NT, BF16>(GRv, rbase + max(c - PF, 0), sw, mow), lane);
            } else {
                a1.load(tile_ptr<NT, BF16>(GRv, rbase + max(c - PF, 0), sw, mow), lane);
            }
            *(floatx4 *)(gwg + c * gstride + (((size_t)sw * NT + mow) * 64 + lane) * 4) = acc;
            if (c == 0) break;
            xch[buf][sw][mow][lane] = acc;
            __syncthreads();
            floatx4 y[2][NT];
            float mx = 0.0f;
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int mo = 0; mo < NT; ++mo) {
                    y[s][mo] = xch[buf][s][mo][lane];
#pragma unroll
                    for (int i = 0; i < 4; ++i) mx = fmaxf(mx, fabsf(y[s][mo][i]));
                }
            buf ^= 1;
            mx = fmaxf(mx, __shfl_xor(mx, 16));
            mx = fmaxf(mx, __shfl_xor(mx, 32));
            const int e = pow2_exponent_f(mx);
            const int su = r > 0 ? prow[c] : 1;
            const double v0 = sfac[c][0] * (su > 0 ? sfac[c][2] : sfac[c][3]);
            const double v1 = sfac[c][1] * (su > 0 ? sfac[c][3] : sfac[c][2]);
            const float m0 = (float)((sw == 0 ? sfac[c][4] : sfac[c][5]) * v0);   // W(s_w,+) v(+)
            const float m1 = (float)((sw == 0 ? sfac[c][5] : sfac[c][4]) * v1);   // W(s_w,-) v(-)
#pragma unroll
            for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    rv[mo][i] = ldexpf(m0 * y[0][mo][i] + m1 * y[1][mo][i], -e);
        }

        __syncthreads();   // every wave's column-0 tile stored before the left sweep reads it

        // ---- left sweep
        floatx4 lam[NT];
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) lam[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        if (grp == 0) lam[0][0] = 1.0f;
        int sprev = 1;
        a0.load(tile_ptr<NT, BF16>(GLv, rbase, sw, mow), lane);
        a1.load(tile_ptr<NT, BF16>(GLv, rbase + min(1, Lx - 1), sw, mow), lane);
        if constexpr (PF == 3) a2.load(tile_ptr<NT, BF16>(GLv, rbase + min(2, Lx - 1), sw, mow), lane);
        floatx4 gc[2][NT], gn[2][NT];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int mo = 0; mo < NT; ++mo) {
                gc[s][mo] = *(const floatx4 *)(gwg + (((size_t)s * NT + mo) * 64 + lane) * 4);
                gn[s][mo] = *(const floatx4 *)(gwg + min(1, Lx - 1) * gstride +
                                               (((size_t)s * NT + mo) * 64 + lane) * 4);
            }
        for (int c = 0; c < Lx; ++c) {
            float d0 = 0.0f, d1 = 0.0f;
#pragma unroll
            for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    d0 = fmaf(lam[mo][i], gc[0][mo][i], d0);
                    d1 = fmaf(lam[mo][i], gc[1][mo][i], d1);
                }
            {
                const float *gp = gwg + min(c + 2, Lx - 1) * gstride;
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int mo = 0; mo < NT; ++mo) {
                        gc[s][mo] = gn[s][mo];
                        gn[s][mo] = *(const floatx4 *)(gp + (((size_t)s * NT + mo) * 64 + lane) * 4);
                    }
            }
            d0 += __shfl_xor(d0, 16);
            d0 += __shfl_xor(d0, 32);
            d1 += __shfl_xor(d1, 16);
            d1 += __shfl_xor(d1, 32);
            const int su = r > 0 ? prow[c] : 1;
            double v0 = sfac[c][0] * (su > 0 ? sfac[c][2] : sfac[c][3]);
            double v1 = sfac[c][1] * (su > 0 ? sfac[c][3] : sfac[c][2]);
            if (c > 0) {
                v0 *= sprev > 0 ? sfac[c][4] : sfac[c][5];
                v1 *= sprev > 0 ? sfac[c][5] : sfac[c][4];
            }
            double w0 = v0 * (double)d0, w1 = v1 * (double)d1;
            if (w0 < 0.0) {
                w0 = 0.0;
                if (leader) atomicAdd(&counters[CNT_CLAMPS], 1ull);
            }
            if (w1 < 0.0) {
                w1 = 0.0;
                if (leader) atomicAdd(&counters[CNT_CLAMPS], 1ull);
            }
            const double tot = w0 + w1;
            const bool bad = !(tot > 0.0 && tot <= 1.79e308);
            if (bad && leader) atomicAdd(&counters[CNT_BOTH], 1ull);
            const double p = bad ? 0.5 : w0 / tot;
            int s;
            if (eval) {
                s = valid ? S[((size_t)b * Ly + r) * Lx + c] : 1;
            } else {
                const int i = r * Lx + c;
                if ((i >> 2) != blk_id) {
                    blk_id = i >> 2;
                    blk = tn_philox(make_uint4((uint32_t)blk_id, (uint32_t)(first_id + b), step,
                                               (inst << 2) | 0u),
                                    k0, k1);
                }
                const double u = tn_u01(tn_word(blk, i & 3));
                s = (u < p) ? 1 : -1;
                if (leader) {
                    S[((size_t)b * Ly + r) * Lx + c] = (int8_t)s;
                    if (fabs(u - p) < 1e-6) atomicAdd(&counters[CNT_NEAR], 1ull);
                }
            }
            if (w == 0 && grp == 0) crow[c] = (int8_t)s;
            {
                int e2;
                mant = frexp(mant * (s > 0 ? p : 1.0 - p), &e2);
                mexp += e2;
            }
            if (h) E -= scpl[c][0] * s;
            if (c > 0) E -= scpl[c][1] * (double)(sprev * s);
            if (r > 0) E -= scpl[c][2] * (double)(su * s);

            const floatx4 acc = a0.mul(lam);
            a0 = a1;
            if constexpr (PF == 3) {
                a1 = a2;
                a2.load(tile_ptr<NT, BF16>(GLv, rbase + min(c + PF, Lx - 1), sw, mow), lane);
            } else {
                a1.load(tile_ptr<NT, BF16>(GLv, rbase + min(c + PF, Lx - 1), sw, mow), lane);
            }
            xch[buf][sw][mow][lane] = acc;
            __syncthreads();
            float mx = 0.0f;
#pragma unroll
            for (int mo = 0; mo < NT; ++mo) {
                lam[mo] = s > 0 ? xch[buf][0][mo][lane] : xch[buf][1][mo][lane];
#pragma unroll
                for (int i = 0; i < 4; ++i) mx = fmaxf(mx, fabsf(lam[mo][i]));
            }
            buf ^= 1;
            mx = fmaxf(mx, __shfl_xor(mx, 16));
            mx = fmaxf(mx, __shfl_xor(mx, 32));
            const int e = pow2_exponent_f(mx);
#pragma unroll
            for (int mo = 0; mo < NT; ++mo)
#pragma unroll
                for (int i = 0; i < 4; ++i) lam[mo][i] = ldexpf(lam[mo][i], -e);
            sprev = s;
        }
        __syncthreads();   // row r spins and factors consumed before row r+1 overwrites
    }
    if (leader) {
        logq[b] = log(mant) + (double)mexp * 0.69314718055994530942;
        energy[b] = E;
    }
}

template <int NT, bool BF16>
int launch_mfma(tn_ctx *ctx, int B, int8_t *S, bool eval, double *logq, double *energy,
                float *g, uint64_t seed, uint64_t step, uint64_t first_id) {
    const int blocks = (B + 15) / 16;
    const void *GR = BF16 ? (const void *)ctx->G16R : (const void *)ctx->G32R;
    const void *GL = BF16 ? (const void *)ctx->G16L : (const void *)ctx->G32L;
    hipLaunchKernelGGL((k_sampler_mfma<NT, BF16>), dim3(blocks), dim3(128 * NT), 0, ctx->stream,
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
    const size_t need = (size_t)blocks * ctx->Lx * 2 * (ctx->Dp / 16) * 64 * 4 * sizeof(float);
    int rc;
    if ((rc = tn_ensure(ctx, &ctx->gscr, &ctx->gscr_cap, need))) return rc;
    float *g = (float *)ctx->gscr;
    if (ctx->prec == TN_BF16)
        return dispatch_nt<true>(ctx, batch, spins, eval, logq, energy, g, seed, step, first_id);
    return dispatch_nt<false>(ctx, batch, spins, eval, logq, energy, g, seed, step, first_id);
}
