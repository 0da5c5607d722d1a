// Metropolis-Hastings acceptance of Algorithm 1 with the tensor-network prior
// g(w'|w) = q(w') (Eqs. mh-acc, tns-prior): chain j accepts its proposal iff
//     u < exp(min(0, (ln q(w) - ln q(w')) - beta (H(w') - H(w))))
// with u = Philox4x32-10(seed; 0, j, step, inst<<2 | 1) word 0 in (0,1), and
// then copies the proposal into its state.  One workgroup per chain; the MH
// step is the given one plus the context's device step base.
#include "common.hpp"

namespace {

__device__ __forceinline__ void accept_body(const tn_acc_desc &A, int j, uint32_t k0, uint32_t k1,
                                            uint32_t step) {
    __shared__ int acc;
    if (threadIdx.x == 0) {
        const double la = (A.slogq[j] - A.plogq[j]) - A.beta * (A.pE[j] - A.sE[j]);
        const uint4 x = tn_philox(make_uint4(0u, (uint32_t)j, step, (A.inst << 2) | 1u), k0, k1);
        const double u = tn_u01(x.x);
        const int a = u < exp(fmin(0.0, la)) ? 1 : 0;
        acc = a;
        A.accepted[j] = (uint8_t)a;
        if (a) {
            A.slogq[j] = A.plogq[j];
            A.sE[j] = A.pE[j];
            atomicAdd(&A.counters[CNT_ACCEPTED], 1ull);
        }
        atomicAdd(&A.counters[CNT_PROPOSED], 1ull);
    }
    __syncthreads();
    if (acc) {
        const int8_t *src = A.pspins + (size_t)j * A.nsite;
        int8_t *dst = A.sspins + (size_t)j * A.nsite;
        for (int t = threadIdx.x; t < A.nsite; t += blockDim.x) dst[t] = src[t];
    }
}

__global__ void __launch_bounds__(256)
k_accept(tn_acc_desc A, uint32_t k0, uint32_t k1, uint64_t step,
         const uint64_t *__restrict__ step_base) {
    accept_body(A, blockIdx.x, k0, k1, (uint32_t)(step + *step_base));
}

// Several instances: instance i owns the blocks (chains) from descs[i].blk0 on.
__global__ void __launch_bounds__(256)
k_accept_multi(const tn_acc_desc *__restrict__ descs, int n, uint32_t k0, uint32_t k1,
               uint64_t step, const uint64_t *__restrict__ step_base) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].blk0 <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const tn_acc_desc A = descs[lo];
    accept_body(A, (int)blockIdx.x - A.blk0, k0, k1, (uint32_t)(step + *step_base));
}

}  // namespace

int tn_launch_accept(tn_ctx *ctx, int chains, uint64_t seed, uint64_t step,
                     const int8_t *prop_spins, const double *prop_logq,
                     const double *prop_energy, int8_t *state_spins, double *state_logq,
                     double *state_energy, uint8_t *accepted) {
    if (chains == 0) return TN_OK;
    tn_acc_desc A;
    A.chains = chains;
    A.nsite = ctx->Lx * ctx->Ly;
    A.beta = ctx->beta;
    A.inst = (uint32_t)ctx->inst;
    A.blk0 = 0;
    A.pspins = prop_spins;
    A.plogq = prop_logq;
    A.pE = prop_energy;
    A.sspins = state_spins;
    A.slogq = state_logq;
    A.sE = state_energy;
    A.accepted = accepted;
    A.counters = ctx->counters;
    hipLaunchKernelGGL(k_accept, dim3(chains), dim3(256), 0, ctx->stream, A, (uint32_t)seed,
                       (uint32_t)(seed >> 32), step, ctx->dstep);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}

int tn_launch_accept_multi(tn_ctx *ctx, const tn_acc_desc *descs, int n, int total_chains,
                           uint64_t seed, uint64_t step) {
    if (total_chains == 0) return TN_OK;
    hipLaunchKernelGGL(k_accept_multi, dim3(total_chains), dim3(256), 0, ctx->stream, descs, n,
                       (uint32_t)seed, (uint32_t)(seed >> 32), step, ctx->dstep);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}
