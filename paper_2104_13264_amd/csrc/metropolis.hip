// Single-spin-flip Metropolis sweeps of the chains' states, to be interleaved
// with TNMH steps (Sec. 3: spin-flip sweeps between TNMH moves help chains that
// the approximate prior alone leaves stuck in frustrated or disordered
// instances).
//
// A sweep visits every site once in checkerboard order: first all sites with
// r + c even, then all with r + c odd.  Sites of one colour share no bond, so
// updating them together equals updating them one after the other.  At site i
// with spin s the local field is
//     F = h_i + J_left s_left + J_right s_right + J_up s_up + J_down s_down
// (summed in this order; missing neighbours of the open boundary add nothing),
// flipping changes the energy of Eq. (ising) by dE = 2 s F, and the flip is
// accepted iff u < exp(-(beta dE)), i.e. with probability min(1, exp(-beta dE)).
// u is word i % 4 of Philox4x32-10 at counter (sweep * 2^14 + i / 4, chain,
// step, inst << 2 | 2), mapped to (x + 1/2) 2^-32.  No product is fused into a
// sum, so the decision is the one the same FP64 expressions give anywhere.
#include "common.hpp"

#pragma clang fp contract(off)

namespace {

constexpr int MT = 256;   // threads per chain

// One workgroup per chain: its spins in LDS for all of its sweeps.
__global__ void __launch_bounds__(MT) k_metropolis(int Lx, int Ly, int nsweeps, double beta,
                                                   const double *__restrict__ Jh,
                                                   const double *__restrict__ Jv,
                                                   const double *__restrict__ h, int8_t *__restrict__ S,
                                                   uint32_t k0, uint32_t k1, uint32_t step, uint32_t inst,
                                                   unsigned long long *__restrict__ counters) {
    extern __shared__ int8_t sp[];   // [Ly][Lx]
    const int chain = blockIdx.x;
    const int nsite = Lx * Ly;
    int8_t *g = S + (size_t)chain * nsite;
    for (int i = threadIdx.x; i < nsite; i += MT) sp[i] = g[i];
    __syncthreads();
    uint32_t flips = 0;
    const int nblk = (nsite + 3) >> 2;
    for (int k = 0; k < nsweeps; ++k) {
        for (int colour = 0; colour < 2; ++colour) {
            for (int b = threadIdx.x; b < nblk; b += MT) {
                const uint4 w = tn_philox(make_uint4(((uint32_t)k << 14) | (uint32_t)b, (uint32_t)chain, step,
                                                     (inst << 2) | 2u),
                                          k0, k1);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = 4 * b + q;
                    if (i >= nsite) break;
                    const int r = i / Lx, c = i - r * Lx;
                    if (((r + c) & 1) != colour) continue;
                    const double s = sp[i];
                    double F = h ? h[i] : 0.0;
                    if (c > 0) F = F + Jh[(size_t)r * (Lx - 1) + c - 1] * (double)sp[i - 1];
                    if (c < Lx - 1) F = F + Jh[(size_t)r * (Lx - 1) + c] * (double)sp[i + 1];
                    if (r > 0) F = F + Jv[(size_t)(r - 1) * Lx + c] * (double)sp[i - Lx];
                    if (r < Ly - 1) F = F + Jv[(size_t)r * Lx + c] * (double)sp[i + Lx];
                    const double dE = (2.0 * s) * F;
                    const double u = tn_u01(tn_word(w, q));
                    if (u < exp(-(beta * dE))) {
                        sp[i] = (int8_t)(-sp[i]);
                        ++flips;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < nsite; i += MT) g[i] = sp[i];
    if (flips) atomicAdd(&counters[CNT_FLIPS], (unsigned long long)flips);
}

}  // namespace

int tn_launch_metropolis(tn_ctx *ctx, int chains, int nsweeps, uint64_t seed, uint64_t step, int8_t *spins) {
    const int nsite = ctx->Lx * ctx->Ly;
    hipLaunchKernelGGL(k_metropolis, dim3(chains), dim3(MT), (size_t)nsite, ctx->stream, ctx->Lx, ctx->Ly,
                       nsweeps, ctx->beta, ctx->Jh, ctx->Jv, ctx->h, spins, (uint32_t)seed,
                       (uint32_t)(seed >> 32), (uint32_t)step, (uint32_t)ctx->inst, ctx->counters);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}
