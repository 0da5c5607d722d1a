// Link overlap of configuration pairs, the replica estimate of
// sum_<ij> <s_i s_j>^2 in the equilibration test of Sec. 3, Eq. (Delta):
//     q[k] = sum over the bonds <ij> of a_i a_j b_i b_j.
// On a periodic lattice the wrapping bonds count too.  One workgroup per pair;
// the sum is an exact integer.
#include "common.hpp"

namespace {

constexpr int QT = 256;

__global__ void __launch_bounds__(QT) k_link_overlap(int Lx, int Ly, int wx, int wy, const int8_t *__restrict__ A,
                                                     const int8_t *__restrict__ B, int32_t *__restrict__ q) {
    __shared__ int part[QT / 64];
    const int nsite = Lx * Ly;
    const int8_t *a = A + (size_t)blockIdx.x * nsite;
    const int8_t *b = B + (size_t)blockIdx.x * nsite;
    int sum = 0;
    for (int i = threadIdx.x; i < nsite; i += QT) {
        const int r = i / Lx, c = i - r * Lx;
        const int ab = (int)a[i] * (int)b[i];
        if (c + 1 < Lx) sum += ab * (int)a[i + 1] * (int)b[i + 1];
        else if (wx) sum += ab * (int)a[i + 1 - Lx] * (int)b[i + 1 - Lx];
        if (r + 1 < Ly) sum += ab * (int)a[i + Lx] * (int)b[i + Lx];
        else if (wy) sum += ab * (int)a[c] * (int)b[c];
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < QT / 64; ++w) t += part[w];
        q[blockIdx.x] = t;
    }
}

}  // namespace

int tn_launch_link_overlap_lattice(tn_ctx *ctx, int Lx, int Ly, int wx, int wy, int n, const int8_t *a,
                                   const int8_t *b, int32_t *q) {
    hipLaunchKernelGGL(k_link_overlap, dim3(n), dim3(QT), 0, ctx->stream, Lx, Ly, wx, wy, a, b, q);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}

int tn_launch_link_overlap(tn_ctx *ctx, int n, const int8_t *a, const int8_t *b, int32_t *q) {
    return tn_launch_link_overlap_lattice(ctx, ctx->Lx, ctx->Ly, 0, 0, n, a, b, q);
}
