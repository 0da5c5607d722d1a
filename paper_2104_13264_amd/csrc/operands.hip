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
// The fp64 tiles (v_mfma_f64_16x16x4f64) follow that instruction's output
// layout, where register i of lane l holds row (l/16) + 4 i of the tile: chunk
// q = 4*mt + i covers rows 16*mt + 4*i .. 16*mt + 4*i + 3 of the next
// product's input, so lane -> row 16*mo + lane%16, col 16*mt + 4*i + lane/16,
// a lane's four chunks of one (mo, mt) in 32 contiguous bytes.
//
// Boltzmann factors, per (r, c):  fac[r][c][0..5] =
//   exp(+-beta h_rc), exp(+-beta Jv_{r-1,c}), exp(+-beta Jh_{r,c-1})
// (1 where the bond or the field is absent).
#include "common.hpp"

#pragma clang fp contract(off)

namespace {

__device__ __forceinline__ uint16_t tn_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Operands of site (r, c) of one instance; gsh: LDS [2][Dp][Dp].
__device__ void ops_site(const tn_ops_desc &O, int r, int c, double *gsh) {
    const int Lx = O.Lx, Ly = O.Ly, D = O.D, Dp = O.Dp;
    const bool last = (r == Ly - 1);
    const int Dl = last ? 1 : O.dims[(r + 1) * (Lx + 1) + c];
    const int Dr = last ? 1 : O.dims[(r + 1) * (Lx + 1) + c + 1];
    const double K = last ? 0.0 : O.beta * O.Jv[r * Lx + c];
    const double *E = O.env + ((size_t)(r + 1) * Lx + c) * 2 * D * D;
    for (int t = threadIdx.x; t < 2 * Dp * Dp; t += blockDim.x) {
        const int s = t / (Dp * Dp), a = (t / Dp) % Dp, b = t % Dp;
        double g = 0.0;
        if (a < Dl && b < Dr) {
            if (last)
                g = 1.0;
            else
                g = fma(tn_pleg(K, s, 0), E[a * 2 * D + b], tn_pleg(K, s, 1) * E[a * 2 * D + D + b]);
        }
        gsh[t] = g;
    }
    __syncthreads();
    const size_t site = (size_t)r * Lx + c;
    if (O.G64r) {
        for (int t = threadIdx.x; t < 2 * D * D; t += blockDim.x) {
            const int s = t / (D * D), a = (t / D) % D, b = t % D;
            O.G64r[site * 2 * D * D + t] = gsh[(s * Dp + a) * Dp + b];
            O.G64c[site * 2 * D * D + (s * D + b) * D + a] = gsh[(s * Dp + a) * Dp + b];
        }
    }
    const int NT = Dp / 16;
    if (O.G32R) {
        // [s][mo][mt][lane][i]: lane holds k-chunks q = 4 mt + i (i = 0..3) of
        // output block mo, 16 contiguous bytes
        for (int t = threadIdx.x; t < 2 * Dp * Dp; t += blockDim.x) {
            const int i = t & 3, lane = (t >> 2) & 63, mt = (t >> 8) % NT, mo = (t >> 8) / NT % NT;
            const int s = t / (Dp * Dp);
            const int row = 16 * mo + (lane & 15), col = 16 * mt + 4 * (lane >> 4) + i;
            O.G32R[site * 2 * Dp * Dp + t] = (float)gsh[(s * Dp + row) * Dp + col];
            O.G32L[site * 2 * Dp * Dp + t] = (float)gsh[(s * Dp + col) * Dp + row];
        }
    }
    if (O.G64MR) {
        for (int t = threadIdx.x; t < 2 * Dp * Dp; t += blockDim.x) {
            const int i = t & 3, lane = (t >> 2) & 63, mt = (t >> 8) % NT, mo = (t >> 8) / NT % NT;
            const int s = t / (Dp * Dp);
            const int row = 16 * mo + (lane & 15), col = 16 * mt + 4 * i + (lane >> 4);
            O.G64MR[site * 2 * Dp * Dp + t] = gsh[(s * Dp + row) * Dp + col];
            O.G64ML[site * 2 * Dp * Dp + t] = gsh[(s * Dp + col) * Dp + row];
        }
    }
    if (O.G16R) {
        // one 16x16x16 chunk per (mo, mt): lane holds 4 consecutive k values
        for (int t = threadIdx.x; t < 2 * Dp * Dp; t += blockDim.x) {
            const int i = t & 3, lane = (t >> 2) & 63, mt = (t >> 8) % NT, mo = (t >> 8) / NT % NT;
            const int s = t / (Dp * Dp);
            const int row = 16 * mo + (lane & 15), col = 16 * mt + 4 * (lane >> 4) + i;
            O.G16R[site * 2 * Dp * Dp + t] = tn_bf16_rne((float)gsh[(s * Dp + row) * Dp + col]);
            O.G16L[site * 2 * Dp * Dp + t] = tn_bf16_rne((float)gsh[(s * Dp + col) * Dp + row]);
        }
    }
}

// Boltzmann factors of site t = r Lx + c of one instance.
__device__ void factor_site(const tn_ops_desc &O, int t) {
    const int Lx = O.Lx;
    const int r = t / Lx, c = t % Lx;
    const double beta = O.beta;
    const double ah = O.h ? beta * O.h[t] : 0.0;
    const double av = r > 0 ? beta * O.Jv[(r - 1) * Lx + c] : 0.0;
    const double aj = c > 0 ? beta * O.Jh[r * (Lx - 1) + c - 1] : 0.0;
    double *f = O.fac + (size_t)t * 6;
    f[0] = exp(ah);
    f[1] = exp(-ah);
    f[2] = exp(av);
    f[3] = exp(-av);
    f[4] = exp(aj);
    f[5] = exp(-aj);
}

__global__ void __launch_bounds__(256) k_make_ops(tn_ops_desc O) {
    extern __shared__ double gsh[];   // [2][Dp][Dp]
    ops_site(O, blockIdx.y, blockIdx.x, gsh);
}

// Instance blockIdx.z of n; the grid covers the widest and tallest lattice.
__global__ void __launch_bounds__(256) k_make_ops_many(const tn_ops_desc *__restrict__ descs) {
    extern __shared__ double gsh[];
    const tn_ops_desc O = descs[blockIdx.z];
    if ((int)blockIdx.x >= O.Lx || (int)blockIdx.y >= O.Ly) return;
    ops_site(O, blockIdx.y, blockIdx.x, gsh);
}

__global__ void __launch_bounds__(256) k_make_factors(tn_ops_desc O) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < O.Lx * O.Ly) factor_site(O, t);
}

__global__ void __launch_bounds__(256) k_make_factors_many(const tn_ops_desc *__restrict__ descs) {
    const tn_ops_desc O = descs[blockIdx.y];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < O.Lx * O.Ly) factor_site(O, t);
}

}  // namespace

tn_ops_desc tn_ops_desc_of(const tn_ctx *ctx, int prec) {
    tn_ops_desc O;
    O.Lx = ctx->Lx;
    O.Ly = ctx->Ly;
    O.D = ctx->D;
    O.Dp = ((ctx->D + 15) / 16) * 16;
    O.beta = ctx->beta;
    O.Jh = ctx->Jh;
    O.Jv = ctx->Jv;
    O.h = ctx->h;
    O.env = ctx->env;
    O.dims = ctx->dims;
    O.fac = ctx->fac;
    O.G64r = prec == TN_FP64 ? ctx->G64r : nullptr;
    O.G64c = prec == TN_FP64 ? ctx->G64c : nullptr;
    O.G32R = prec == TN_FP32 ? ctx->G32R : nullptr;
    O.G32L = prec == TN_FP32 ? ctx->G32L : nullptr;
    O.G16R = prec == TN_BF16 ? ctx->G16R : nullptr;
    O.G16L = prec == TN_BF16 ? ctx->G16L : nullptr;
    O.G64MR = prec == TN_FP64_MFMA ? ctx->G64MR : nullptr;
    O.G64ML = prec == TN_FP64_MFMA ? ctx->G64ML : nullptr;
    return O;
}

int tn_make_operands(tn_ctx *ctx, int prec) {
    const int Lx = ctx->Lx, Ly = ctx->Ly, D = ctx->D;
    const int Dp = ((D + 15) / 16) * 16;
    ctx->Dp = Dp;
    int rc;
    const size_t sites = (size_t)Lx * Ly;
    if ((rc = tn_ensure(ctx, (void **)&ctx->fac, &ctx->fac_cap, sites * 6 * sizeof(double))))
        return rc;
    if (prec == TN_FP64) {
        const size_t n = sites * 2 * D * D;
        if ((rc = tn_ensure(ctx, (void **)&ctx->G64r, &ctx->ops_cap64, 2 * n * sizeof(double))))
            return rc;
        ctx->G64c = ctx->G64r + n;
    } else if (prec == TN_FP32) {
        const size_t n = sites * 2 * Dp * Dp;
        if ((rc = tn_ensure(ctx, (void **)&ctx->G32R, &ctx->ops_cap32, 2 * n * sizeof(float))))
            return rc;
        ctx->G32L = ctx->G32R + n;
    } else if (prec == TN_FP64_MFMA) {
        if (Dp > 32) return tn_fail(ctx, TN_EINVAL, "the batched fp64 sampler supports D <= 32");
        const size_t n = sites * 2 * Dp * Dp;
        if ((rc = tn_ensure(ctx, (void **)&ctx->G64MR, &ctx->ops_cap64m, 2 * n * sizeof(double))))
            return rc;
        ctx->G64ML = ctx->G64MR + n;
    } else {
        const size_t n = sites * 2 * Dp * Dp;
        if ((rc = tn_ensure(ctx, (void **)&ctx->G16R, &ctx->ops_cap16, 2 * n * sizeof(uint16_t))))
            return rc;
        ctx->G16L = ctx->G16R + n;
    }
    const tn_ops_desc O = tn_ops_desc_of(ctx, prec);
    hipLaunchKernelGGL(k_make_factors, dim3((unsigned)((sites + 255) / 256)), dim3(256), 0, ctx->stream, O);
    TN_HIP(ctx, hipGetLastError());
    const size_t lds = (size_t)2 * Dp * Dp * sizeof(double);
    TN_HIP(ctx, hipFuncSetAttribute((const void *)k_make_ops,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_make_ops, dim3(Lx, Ly), dim3(256), lds, ctx->stream, O);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}

int tn_make_operands_many(tn_ctx *ctx, const tn_ops_desc *descs, int n, int maxLx, int maxLy, int maxDp) {
    if (n <= 0) return TN_OK;
    const size_t sites = (size_t)maxLx * maxLy;
    const size_t lds = (size_t)2 * maxDp * maxDp * sizeof(double);
    TN_HIP(ctx, hipFuncSetAttribute((const void *)k_make_ops_many,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    constexpr int CHUNK = 32768;   // instances per launch (grid y / z limit)
    for (int base = 0; base < n; base += CHUNK) {
        const int m = n - base < CHUNK ? n - base : CHUNK;
        hipLaunchKernelGGL(k_make_factors_many, dim3((unsigned)((sites + 255) / 256), m), dim3(256), 0,
                           ctx->stream, descs + base);
        hipLaunchKernelGGL(k_make_ops_many, dim3(maxLx, maxLy, m), dim3(256), lds, ctx->stream, descs + base);
        TN_HIP(ctx, hipGetLastError());
    }
    return TN_OK;
}
