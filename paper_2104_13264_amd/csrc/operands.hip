// Sampler operands derived from the fp64 environment stack.
//
// For row r the rows below are env r+1 (trivial for the last row).  The site
// (r,c) with spin s couples to it through the down leg of its vertical bond,
//     G_c(s)[a][b] = sum_d P(s,d) env_{r+1,c}[a][d][b]      (App. A split)
// so that the row contraction of the sampler is a product of these matrices
// with the horizontal bond weights and the field / fixed-neighbour factors.
//
// Stored forms, per (r, c, s):
//   G64r  [a][b]  and  G64c [b][a]          fp64, D x D   (plain path)
//   G32R, G32L                              fp32 MFMA A-operand tiles of G and
//   G16R, G16L                              G^T (bf16 for the bf16 path)
// Tile layout for v_mfma_f32_16x16x4f32 with padded bond Dp = 16*NT:
//   index (((((r*Lx + c)*2 + s)*NT + mo)*NT + mt)*64 + lane)*4 + i,
//   k-chunk q = 4*mt + i, lane -> row 16*mo + lane%16, col 16*mt + 4*(lane/16) + i,
// which makes the k-chunk q of the next product equal to accumulator register
// i of output tile mt, so chained products need no data movement; a lane's
// four chunks of one (mo, mt) are 16 contiguous bytes (one load).
// The bf16 tiles (v_mfma_f32_16x16x16_bf16) use chunk q = mt, lane -> row
// 16*mo + lane%16, cols 16*mt + 4*(lane/16) + i for i = 0..3 packed in 8 bytes.
//
// Boltzmann factors, per (r, c):  fac[r][c][0..5] =
//   exp(+-beta h_rc), exp(+-beta Jv_{r-1,c}), exp(+-beta Jh_{r,c-1})
// (1 where the bond or the field is absent).
#include "common.hpp"

namespace {

__device__ __forceinline__ uint16_t tn_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ void __launch_bounds__(256)
k_make_ops(int Lx, int Ly, int D, int Dp, double beta, const double *__restrict__ Jv,
           const double *__restrict__ env, const int *__restrict__ dims,
           double *__restrict__ G64r, double *__restrict__ G64c, float *__restrict__ G32R,
           float *__restrict__ G32L, uint16_t *__restrict__ G16R, uint16_t *__restrict__ G16L) {
    extern __shared__ double gsh[];   // [2][Dp][Dp]
    const int c = blockIdx.x, r = blockIdx.y;
    const bool last = (r == Ly - 1);
    const int Dl = last ? 1 : dims[(r + 1) * (Lx + 1) + c];
    const int Dr = last ? 1 : dims[(r + 1) * (Lx + 1) + c + 1];
    const double K = last ? 0.0 : beta * Jv[r * Lx + c];
    const double *E = env + ((size_t)(r + 1) * Lx + c) * 2 * D * D;
    for (int t = threadIdx.x; t < 2 * Dp * Dp; t += blockDim.x) {
        const int s = t / (Dp * Dp), a = (t / Dp) % Dp, b = t % Dp;
        double g = 0.0;
        if (a < Dl && b < Dr) {
            if (last)
                g = 1.0;
            else
                g = tn_pleg(K, s, 0) * E[a * 2 * D + b] + tn_pleg(K, s, 1) * E[a * 2 * D + D + b];
        }
        gsh[t] = g;
    }
    __syncthreads();
    const size_t site = (size_t)r * Lx + c;
    if (G64r) {
        for (int t = threadIdx.x; t < 2 * D * D; t += blockDim.x) {
            const int s = t / (D * D), a = (t / D) % D, b = t % D;
            G64r[site * 2 * D * D + t] = gsh[(s * Dp + a) * Dp + b];
            G64c[site * 2 * D * D + (s * D + b) * D + a] = gsh[(s * Dp + a) * Dp + b];
        }
    }
    const int NT = Dp / 16;
    if (G32R) {
        // [s][mo][mt][lane][i]: lane holds k-chunks q = 4 mt + i (i = 0..3) of
        // output block mo, 16 contiguous bytes
        for (int t = threadIdx.x; t < 2 * Dp * Dp; t += blockDim.x) {
            const int i = t & 3, lane = (t >> 2) & 63, mt = (t >> 8) % NT, mo = (t >> 8) / NT % NT;
            const int s = t / (Dp * Dp);
            const int row = 16 * mo + (lane & 15), col = 16 * mt + 4 * (lane >> 4) + i;
            G32R[site * 2 * Dp * Dp + t] = (float)gsh[(s * Dp + row) * Dp + col];
            G32L[site * 2 * Dp * Dp + t] = (float)gsh[(s * Dp + col) * Dp + row];
        }
    }
    if (G16R) {
        // one 16x16x16 chunk per (mo, mt): lane holds 4 consecutive k values
        for (int t = threadIdx.x; t < 2 * Dp * Dp; t += blockDim.x) {
            const int i = t & 3, lane = (t >> 2) & 63, mt = (t >> 8) % NT, mo = (t >> 8) / NT % NT;
            const int s = t / (Dp * Dp);
            const int row = 16 * mo + (lane & 15), col = 16 * mt + 4 * (lane >> 4) + i;
            G16R[site * 2 * Dp * Dp + t] = tn_bf16_rne((float)gsh[(s * Dp + row) * Dp + col]);
            G16L[site * 2 * Dp * Dp + t] = tn_bf16_rne((float)gsh[(s * Dp + col) * Dp + row]);
        }
    }
}

__global__ void k_make_factors(int Lx, int Ly, double beta, const double *__restrict__ Jh,
                               const double *__restrict__ Jv, const double *__restrict__ h,
                               double *__restrict__ fac) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Lx * Ly) return;
    const int r = t / Lx, c = t % Lx;
    const double ah = h ? beta * h[t] : 0.0;
    const double av = r > 0 ? beta * Jv[(r - 1) * Lx + c] : 0.0;
    const double aj = c > 0 ? beta * Jh[r * (Lx - 1) + c - 1] : 0.0;
    double *f = fac + (size_t)t * 6;
    f[0] = exp(ah);
    f[1] = exp(-ah);
    f[2] = exp(av);
    f[3] = exp(-av);
    f[4] = exp(aj);
    f[5] = exp(-aj);
}

}  // namespace

int tn_make_factors(tn_ctx *ctx, double *fac);

int tn_make_operands(tn_ctx *ctx, int prec) {
    const int Lx = ctx->Lx, Ly = ctx->Ly, D = ctx->D;
    const int Dp = ((D + 15) / 16) * 16;
    ctx->Dp = Dp;
    int rc;
    const size_t sites = (size_t)Lx * Ly;
    if ((rc = tn_ensure(ctx, (void **)&ctx->fac, &ctx->fac_cap, sites * 6 * sizeof(double))))
        return rc;
    if ((rc = tn_make_factors(ctx, ctx->fac))) return rc;
    double *G64r = nullptr, *G64c = nullptr;
    float *G32R = nullptr, *G32L = nullptr;
    uint16_t *G16R = nullptr, *G16L = nullptr;
    if (prec == TN_FP64) {
        const size_t n = sites * 2 * D * D;
        if ((rc = tn_ensure(ctx, (void **)&ctx->G64r, &ctx->ops_cap64, 2 * n * sizeof(double))))
            return rc;
        ctx->G64c = ctx->G64r + n;
        G64r = ctx->G64r;
        G64c = ctx->G64c;
    } else if (prec == TN_FP32) {
        const size_t n = sites * 2 * Dp * Dp;
        if ((rc = tn_ensure(ctx, (void **)&ctx->G32R, &ctx->ops_cap32, 2 * n * sizeof(float))))
            return rc;
        ctx->G32L = ctx->G32R + n;
        G32R = ctx->G32R;
        G32L = ctx->G32L;
    } else {
        const size_t n = sites * 2 * Dp * Dp;
        if ((rc = tn_ensure(ctx, (void **)&ctx->G16R, &ctx->ops_cap16, 2 * n * sizeof(uint16_t))))
            return rc;
        ctx->G16L = ctx->G16R + n;
        G16R = ctx->G16R;
        G16L = ctx->G16L;
    }
    const size_t lds = (size_t)2 * Dp * Dp * sizeof(double);
    TN_HIP(ctx, hipFuncSetAttribute((const void *)k_make_ops,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_make_ops, dim3(Lx, Ly), dim3(256), lds, ctx->stream, Lx, Ly, D, Dp,
                       ctx->beta, ctx->Jv, ctx->env, ctx->dims, G64r, G64c, G32R, G32L, G16R,
                       G16L);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}

int tn_make_factors(tn_ctx *ctx, double *fac) {
    const int n = ctx->Lx * ctx->Ly;
    hipLaunchKernelGGL(k_make_factors, dim3((n + 255) / 256), dim3(256), 0, ctx->stream,
                       ctx->Lx, ctx->Ly, ctx->beta, ctx->Jh, ctx->Jv, ctx->h, fac);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}
