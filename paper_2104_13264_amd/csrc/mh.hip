// Metropolis-Hastings acceptance of Algorithm 1 with the tensor-network prior
// g(w'|w) = q(w') (Eqs. mh-acc, tns-prior): chain j accepts its proposal iff
//     u < exp(min(0, (ln q(w) - ln q(w')) - beta (H(w') - H(w))))
// with u = Philox4x32-10(seed; 0, j, step, inst<<2 | 1) word 0 in (0,1), and
// then copies the proposal into its state.  One workgroup per chain.
#include "common.hpp"

namespace {

__global__ void __launch_bounds__(256)
k_accept(int chains, int nsite, double beta, uint32_t k0, uint32_t k1, uint32_t step,
         uint32_t inst, const int8_t *__restrict__ pspins, const double *__restrict__ plogq,
         const double *__restrict__ pE, int8_t *__restrict__ sspins, double *__restrict__ slogq,
         double *__restrict__ sE, uint8_t *__restrict__ accepted,
         unsigned long long *__restrict__ counters) {
    const int j = blockIdx.x;
    __shared__ int acc;
    if (threadIdx.x == 0) {
        const double la = (slogq[j] - plogq[j]) - beta * (pE[j] - sE[j]);
        const uint4 x = tn_philox(make_uint4(0u, (uint32_t)j, step, (inst << 2) | 1u), k0, k1);
        const double u = tn_u01(x.x);
        const int a = u < exp(fmin(0.0, la)) ? 1 : 0;
        acc = a;
        accepted[j] = (uint8_t)a;
        if (a) {
            slogq[j] = plogq[j];
            sE[j] = pE[j];
            atomicAdd(&counters[CNT_ACCEPTED], 1ull);
        }
        atomicAdd(&counters[CNT_PROPOSED], 1ull);
    }
    __syncthreads();
    if (acc) {
        const int8_t *src = pspins + (size_t)j * nsite;
        int8_t *dst = sspins + (size_t)j * nsite;
        for (int t = threadIdx.x; t < nsite; t += blockDim.x) dst[t] = src[t];
    }
}

}  // namespace

int tn_launch_accept(tn_ctx *ctx, int chains, uint64_t seed, uint64_t step,
                     const int8_t *prop_spins, const double *prop_logq,
                     const double *prop_energy, int8_t *state_spins, double *state_logq,
                     double *state_energy, uint8_t *accepted) {
    if (chains == 0) return TN_OK;
    hipLaunchKernelGGL(k_accept, dim3(chains), dim3(256), 0, ctx->stream, chains,
                       ctx->Lx * ctx->Ly, ctx->beta, (uint32_t)seed, (uint32_t)(seed >> 32),
                       (uint32_t)step, (uint32_t)ctx->inst, prop_spins, prop_logq, prop_energy,
                       state_spins, state_logq, state_energy, accepted, ctx->counters);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}
