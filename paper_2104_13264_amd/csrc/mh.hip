// Metropolis-Hastings acceptance of Algorithm 1 with the tensor-network prior
// g(w'|w) = q(w') (Eqs. mh-acc, tns-prior): chain j accepts its proposal iff
//     u < exp(min(0, (ln q(w) - ln q(w')) - beta (H(w') - H(w))))
// with u = Philox4x32-10(seed; 0, j, step, inst<<2 | 1) word 0 in (0,1), and
// then copies the proposal into its state.  A workgroup takes 16 chains; the
// MH step is the given one plus the context's device step base.
#include "common.hpp"

namespace {

constexpr int AC = 16;   // chains per workgroup

// The decision of chain j and its ln q / energy update; 1 if accepted.
__device__ __forceinline__ int accept_one(const tn_acc_desc &A, int j, uint32_t k0, uint32_t k1,
                                          uint32_t step) {
    const double la = (A.slogq[j] - A.plogq[j]) - A.beta * (A.pE[j] - A.sE[j]);
    const uint4 x = tn_philox(make_uint4(0u, (uint32_t)j, step, (A.inst << 2) | 1u), k0, k1);
    const double u = tn_u01(x.x);
    const int a = u < exp(fmin(0.0, la)) ? 1 : 0;
    A.accepted[j] = (uint8_t)a;
    if (a) {
        A.slogq[j] = A.plogq[j];
        A.sE[j] = A.pE[j];
    }
    if (A.eser) A.eser[j] = a ? A.pE[j] : A.sE[j];
    return a;
}

// An accepted proposal's spins into the state, by the whole workgroup:
// 16-byte words when both rows of bytes are aligned to them, else bytes.
__device__ __forceinline__ void copy_spins(const tn_acc_desc &A, int j) {
    const int8_t *src = A.pspins + (size_t)j * A.nsite;
    int8_t *dst = A.sspins + (size_t)j * A.nsite;
    if ((((uintptr_t)src | (uintptr_t)dst | (uintptr_t)A.nsite) & 15) == 0) {
        const uint4 *s4 = (const uint4 *)src;
        uint4 *d4 = (uint4 *)dst;
        for (int t = threadIdx.x; t < (A.nsite >> 4); t += blockDim.x) d4[t] = s4[t];
    } else {
        for (int t = threadIdx.x; t < A.nsite; t += blockDim.x) dst[t] = src[t];
    }
}

// Chains c0 .. c0 + AC - 1 of the launch (c0 = AC blockIdx.x), chain c being
// chain c - blk0 of the last instance whose blk0 <= c: the first AC threads
// decide, thread 0 adds the counts of each instance present with one atomic
// per counter, then all threads copy the accepted chains.
template <bool MULTI>
__device__ __forceinline__ void accept_group(const tn_acc_desc *__restrict__ descs, const tn_acc_desc &A0,
                                             int n, int total, uint32_t k0, uint32_t k1, uint32_t step) {
    __shared__ int acc[AC], ins[AC], jj[AC];
    auto D = [&](int i) -> const tn_acc_desc & {
        if constexpr (MULTI) return descs[i];
        else return A0;
    };
    const int c0 = (int)blockIdx.x * AC;
    if (threadIdx.x < AC) {
        const int c = c0 + (int)threadIdx.x;
        int a = 0, i = -1, j = 0;
        if (c < total) {
            i = 0;
            if constexpr (MULTI) {
                int lo = 0, hi = n - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (descs[mid].blk0 <= c) lo = mid;
                    else hi = mid - 1;
                }
                i = lo;
            }
            j = c - D(i).blk0;
            a = accept_one(D(i), j, k0, k1, step);
        }
        acc[threadIdx.x] = a;
        ins[threadIdx.x] = i;
        jj[threadIdx.x] = j;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int l = 0;
        while (l < AC && ins[l] >= 0) {   // chains of one instance are consecutive
            const int i = ins[l];
            unsigned long long na = 0, np = 0;
            for (; l < AC && ins[l] == i; ++l) {
                na += (unsigned long long)acc[l];
                ++np;
            }
            if (na) atomicAdd(&D(i).counters[CNT_ACCEPTED], na);
            atomicAdd(&D(i).counters[CNT_PROPOSED], np);
        }
    }
    for (int l = 0; l < AC; ++l)
        if (acc[l]) copy_spins(D(ins[l]), jj[l]);
}

__global__ void __launch_bounds__(256)
k_accept(tn_acc_desc A, uint32_t k0, uint32_t k1, uint64_t step,
         const uint64_t *__restrict__ step_base) {
    accept_group<false>(nullptr, A, 1, A.chains, k0, k1, (uint32_t)(step + *step_base));
}

// Several instances: instance i owns the chains from descs[i].blk0 on.
__global__ void __launch_bounds__(256)
k_accept_multi(const tn_acc_desc *__restrict__ descs, int n, int total, uint32_t k0, uint32_t k1,
               uint64_t step, const uint64_t *__restrict__ step_base) {
    accept_group<true>(descs, descs[0], n, total, k0, k1, (uint32_t)(step + *step_base));
}

}  // namespace

int tn_launch_accept(tn_ctx *ctx, int chains, uint64_t seed, uint64_t step,
                     const int8_t *prop_spins, const double *prop_logq,
                     const double *prop_energy, int8_t *state_spins, double *state_logq,
                     double *state_energy, uint8_t *accepted,
                     double *energy_series) {
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
    A.eser = energy_series;
    hipLaunchKernelGGL(k_accept, dim3((chains + AC - 1) / AC), dim3(256), 0, ctx->stream, A, (uint32_t)seed,
                       (uint32_t)(seed >> 32), step, ctx->dstep);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}

int tn_launch_accept_multi(tn_ctx *ctx, const tn_acc_desc *descs, int n, int total_chains,
                           uint64_t seed, uint64_t step) {
    if (total_chains == 0) return TN_OK;
    hipLaunchKernelGGL(k_accept_multi, dim3((total_chains + AC - 1) / AC), dim3(256), 0, ctx->stream, descs,
                       n, total_chains, (uint32_t)seed, (uint32_t)(seed >> 32), step, ctx->dstep);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
}
