// Plain fp64 sampler: the sequential Bayes-chain-rule draw of Sec. 2
// (Eqs. bayes, pi-approx) with the conditionals of App. A Eq. (proba-ratio-apx)
// evaluated against the stored environment, in fp64 vector arithmetic with one
// kernel launch per lattice row.
//
// Work split: a "team" of T lanes (T = smallest power of two >= D) owns one
// proposal; lane j holds component j of the proposal's bond vectors, and the
// matrix-vector products broadcast the input vector across the team with
// lane shuffles.  No LDS is used.
//
// Site order: snake (even rows left to right, odd rows right to left).
// Row r, given the fixed row r-1 above and env r+1 below (rightward row; a
// leftward row is the mirror image with G^T and the bonds to the right):
//   environment sweep (c = Lx-1 .. 0):  y_s = G_c(s) r_s^(c)  (stored per column)
//       r_s'^(c-1) = sum_s W_{c-1,c}(s',s) v_c(s) y_s,   v_c(s) = exp(beta h s)
//       exp(beta Jv s_up s), W = exp(beta Jh s' s); rescaled by a power of two
//   sampling sweep (c = 0 .. Lx-1):   w(s) = v_c(s) hf(s) <Lam, y_s>,
//       hf(s) = exp(beta Jh s_{c-1} s); clamp; p+ = w+/(w+ + w-); draw;
//       ln q += ln p_s;  Lam <- Lam G_c(s), rescaled by a power of two
#include "common.hpp"

namespace {

template <int T>
__device__ __forceinline__ double team_sum(double v) {
#pragma unroll
    for (int m = T / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, T);
    return v;
}
template <int T>
__device__ __forceinline__ double team_max(double v) {
#pragma unroll
    for (int m = T / 2; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, T));
    return v;
}

__device__ __forceinline__ int pow2_exponent(double m) {
    int e = 0;
    if (m > 0.0 && m <= 1.79e308) frexp(m, &e);
    return e;
}

template <int T>
__global__ void __launch_bounds__(256)
k_row_fp64(int r, int B, int Lx, int Ly, int D, const double *__restrict__ Jh,
           const double *__restrict__ Jv, const double *__restrict__ h,
           const double *__restrict__ fac, const int *__restrict__ dims,
           const double *__restrict__ G64r, const double *__restrict__ G64c,
           int8_t *__restrict__ S, int eval, double *__restrict__ logq,
           double *__restrict__ energy, double *__restrict__ gscr, uint32_t k0, uint32_t k1,
           uint64_t first_id, uint64_t step0, const uint64_t *__restrict__ step_base,
           int per_step, uint32_t inst,
           unsigned long long *__restrict__ counters) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = tid / T, j = tid % T;
    if (b >= B) return;   // whole teams leave together (T divides 64)
    const int *dm = dims + (size_t)(r + 1) * (Lx + 1);
    const size_t DD = (size_t)D * D;
    const double *Gr = G64r + (size_t)r * Lx * 2 * DD;
    const double *Gc = G64c + (size_t)r * Lx * 2 * DD;
    const double *fr = fac + (size_t)r * Lx * 6;
    double *gs = gscr + (size_t)b * Lx * 2 * D;
    const int8_t *up = r > 0 ? S + ((size_t)b * Ly + r - 1) * Lx : nullptr;
    int8_t *row = S + ((size_t)b * Ly + r) * Lx;

    const bool rightward = (r & 1) == 0;   // snake order: even rows left to right
    // Full teams with T <= 32 load both spins' operands of a drawing column
    // before the draw and multiply the drawn spin's after it, so that the
    // draw does not wait for their loads (two columns of T doubles leave two
    // waves per SIMD, all that a launch of 4096 proposals fills)
    constexpr bool PIPE = T <= 32;
    constexpr int TP = PIPE ? T : 1;
    const bool pipe = PIPE && D == T;

    // ---- environment sweep of the free columns, from the far end of the row
    double r0 = (j == 0) ? 1.0 : 0.0, r1 = r0;
    for (int t = 0; t < Lx; ++t) {
        const int c = rightward ? Lx - 1 - t : t;
        const int Dl = dm[c], Dr = dm[c + 1];
        const int su = up ? up[c] : 1;   // loaded ahead of the operands
        double y0 = 0.0, y1 = 0.0;
        if (D == T) {
            // full teams: G is zero outside Dl x Dr and so are the vector
            // components past the bond, so a fixed T-term product adds exact
            // zeros after the same terms in the same order; unrolled, its
            // shuffles and loads issue together instead of one chain per term
            const double *G0 = (rightward ? Gc : Gr) + (size_t)c * 2 * DD, *G1 = G0 + DD;
#pragma unroll
            for (int k = 0; k < T; ++k) {
                const double x0 = __shfl(r0, k, T), x1 = __shfl(r1, k, T);
                y0 += G0[k * D + j] * x0;
                y1 += G1[k * D + j] * x1;
            }
        } else if (rightward) {   // y_s = G_c(s) r_s: input right bond, output left bond
            const double *G0 = Gc + (size_t)c * 2 * DD, *G1 = G0 + DD;
            for (int k = 0; k < Dr; ++k) {
                const double x0 = __shfl(r0, k, T), x1 = __shfl(r1, k, T);
                if (j < Dl) {
                    y0 += G0[k * D + j] * x0;
                    y1 += G1[k * D + j] * x1;
                }
            }
        } else {           // y_s = G_c(s)^T l_s: input left bond, output right bond
            const double *G0 = Gr + (size_t)c * 2 * DD, *G1 = G0 + DD;
            for (int k = 0; k < Dl; ++k) {
                const double x0 = __shfl(r0, k, T), x1 = __shfl(r1, k, T);
                if (j < Dr) {
                    y0 += G0[k * D + j] * x0;
                    y1 += G1[k * D + j] * x1;
                }
            }
        }
        if (j < D) {
            gs[(c * 2 + 0) * D + j] = y0;
            gs[(c * 2 + 1) * D + j] = y1;
        }
        if (t + 1 < Lx) {
            const double *f = fr + c * 6;
            // bond towards the next column of the sweep
            const double *fb = fr + (rightward ? c : c + 1) * 6;
            const double v0 = f[0] * (su > 0 ? f[2] : f[3]);   // s = +1
            const double v1 = f[1] * (su > 0 ? f[3] : f[2]);   // s = -1
            const double n0 = fb[4] * v0 * y0 + fb[5] * v1 * y1;
            const double n1 = fb[5] * v0 * y0 + fb[4] * v1 * y1;
            const int e = pow2_exponent(team_max<T>(fmax(fabs(n0), fabs(n1))));
            r0 = ldexp(n0, -e);
            r1 = ldexp(n1, -e);
        }
    }

    // ---- sampling sweep in the row's direction
    double lam = (j == 0) ? 1.0 : 0.0;
    int sprev = 1;
    double lq = 0.0, E = 0.0;
    uint4 blk = make_uint4(0, 0, 0, 0);
    int blk_id = -1;
    for (int t = 0; t < Lx; ++t) {
        const int c = rightward ? t : Lx - 1 - t;
        const int Dl = dm[c], Dr = dm[c + 1];
        const double *f = fr + c * 6;
        const int su = up ? up[c] : 1;
        double v0 = f[0] * (su > 0 ? f[2] : f[3]);
        double v1 = f[1] * (su > 0 ? f[3] : f[2]);
        if (t > 0) {   // bond to the previously drawn neighbour
            const double *fb = fr + (rightward ? c : c + 1) * 6;
            v0 *= sprev > 0 ? fb[4] : fb[5];
            v1 *= sprev > 0 ? fb[5] : fb[4];
        }
        const double g0 = j < D ? gs[(c * 2 + 0) * D + j] : 0.0;
        const double g1 = j < D ? gs[(c * 2 + 1) * D + j] : 0.0;
        double gd0[TP], gd1[TP];   // both spins' operands of the left product
        if (pipe) {
            const double *G0 = (rightward ? Gr : Gc) + (size_t)c * 2 * DD;
#pragma unroll
            for (int a = 0; a < TP; ++a) {
                gd0[a] = G0[a * D + j];
                gd1[a] = G0[DD + a * D + j];
            }
        }
        double w0 = v0 * team_sum<T>(lam * g0);
        double w1 = v1 * team_sum<T>(lam * g1);
        if (w0 < 0.0) {
            w0 = 0.0;
            if (j == 0) atomicAdd(&counters[CNT_CLAMPS], 1ull);
        }
        if (w1 < 0.0) {
            w1 = 0.0;
            if (j == 0) atomicAdd(&counters[CNT_CLAMPS], 1ull);
        }
        const double tot = w0 + w1;
        const bool bad = !(tot > 0.0 && tot <= 1.79e308);
        if (bad && j == 0) atomicAdd(&counters[CNT_BOTH], 1ull);
        const double p = bad ? 0.5 : w0 / tot;
        int s;
        if (eval) {
            s = row[c];
        } else {
            const int i = r * Lx + c;
            if ((i >> 2) != blk_id) {
                blk_id = i >> 2;
                const uint64_t id = first_id + (uint64_t)b % (uint64_t)per_step;
                const uint32_t st = (uint32_t)(step0 + *step_base + (uint64_t)b / (uint64_t)per_step);
                blk = tn_philox(make_uint4((uint32_t)blk_id, (uint32_t)id, st, (inst << 2) | 0u),
                                k0, k1);
            }
            const double u = tn_u01(tn_word(blk, i & 3));
            s = (u < p) ? 1 : -1;
            if (j == 0) {
                row[c] = (int8_t)s;
                if (fabs(u - p) < 1e-6) atomicAdd(&counters[CNT_NEAR], 1ull);
            }
        }
        lq += log(s > 0 ? p : 1.0 - p);
        // energy, Eq. (ising): field, bond to the previous neighbour, bond above
        if (h) E -= h[r * Lx + c] * s;
        if (t > 0) E -= Jh[r * (Lx - 1) + (rightward ? c - 1 : c)] * (double)(sprev * s);
        if (up) E -= Jv[(r - 1) * Lx + c] * (double)(up[c] * s);
        double nl = 0.0;
        if (pipe) {        // the drawn spin's operands, loaded before the draw
#pragma unroll
            for (int a = 0; a < TP; ++a) {
                const double x = __shfl(lam, a, T);
                nl += x * (s > 0 ? gd0[a] : gd1[a]);
            }
        } else if (D == T) {      // as in the sweep: a fixed T-term product
            const double *Gs = (rightward ? Gr : Gc) + ((size_t)c * 2 + (s > 0 ? 0 : 1)) * DD;
#pragma unroll
            for (int a = 0; a < T; ++a) {
                const double x = __shfl(lam, a, T);
                nl += x * Gs[a * D + j];
            }
        } else if (rightward) {   // Lam <- Lam G_c(s): input left bond, output right bond
            const double *Gs = Gr + ((size_t)c * 2 + (s > 0 ? 0 : 1)) * DD;
            for (int a = 0; a < Dl; ++a) {
                const double x = __shfl(lam, a, T);
                if (j < Dr) nl += x * Gs[a * D + j];
            }
        } else {           // Lam <- G_c(s) Lam: input right bond, output left bond
            const double *Gs = Gc + ((size_t)c * 2 + (s > 0 ? 0 : 1)) * DD;
            for (int k = 0; k < Dr; ++k) {
                const double x = __shfl(lam, k, T);
                if (j < Dl) nl += x * Gs[k * D + j];
            }
        }
        const int e = pow2_exponent(team_max<T>(fabs(nl)));
        lam = ldexp(nl, -e);
        sprev = s;
    }
    if (j == 0) {
        if (r == 0) {
            logq[b] = lq;
            energy[b] = E;
        } else {
            logq[b] += lq;
            energy[b] += E;
        }
    }
}

template <int T>
int launch_rows(tn_ctx *ctx, int B, int8_t *S, bool eval, double *logq, double *energy,
                double *gscr, uint64_t seed, uint64_t step0, int per_step, uint64_t first_id) {
    const int threads = 256;
    const size_t total = (size_t)B * T;
    const int blocks = (int)((total + threads - 1) / threads);
    for (int r = 0; r < ctx->Ly; ++r) {
        hipLaunchKernelGGL(k_row_fp64<T>, dim3(blocks), dim3(threads), 0, ctx->stream, r, B,
                           ctx->Lx, ctx->Ly, ctx->D, ctx->Jh, ctx->Jv, ctx->h, ctx->fac,
                           ctx->dims, ctx->G64r, ctx->G64c, S, eval ? 1 : 0, logq, energy,
                           gscr, (uint32_t)seed, (uint32_t)(seed >> 32), first_id, step0,
                           ctx->dstep, per_step, (uint32_t)ctx->inst, ctx->counters);
        TN_HIP(ctx, hipGetLastError());
    }
    return TN_OK;
}

}  // namespace

int tn_run_fp64(tn_ctx *ctx, int batch, uint64_t seed, uint64_t step0, int per_step,
                uint64_t first_id, int8_t *spins, bool eval, double *logq, double *energy,
                void *scr) {
    if (batch == 0) return TN_OK;
    if (per_step <= 0) return tn_fail(ctx, TN_EINVAL, "proposals per step must be positive");
    int rc;
    if (!scr) {
        if ((rc = tn_ensure(ctx, &ctx->gscr, &ctx->gscr_cap, tn_fp64_scratch_bytes(ctx, batch)))) return rc;
        scr = ctx->gscr;
    }
    double *g = (double *)scr;
    int T = 1;
    while (T < ctx->D) T <<= 1;
    switch (T) {
    case 1: return launch_rows<1>(ctx, batch, spins, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 2: return launch_rows<2>(ctx, batch, spins, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 4: return launch_rows<4>(ctx, batch, spins, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 8: return launch_rows<8>(ctx, batch, spins, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 16: return launch_rows<16>(ctx, batch, spins, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 32: return launch_rows<32>(ctx, batch, spins, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 64: return launch_rows<64>(ctx, batch, spins, eval, logq, energy, g, seed, step0, per_step, first_id);
    default: return tn_fail(ctx, TN_EINVAL, "bond dimension above 64");
    }
}
