// Boundary-MPS environments of the 2D Ising network (App. A): for every row
// k = Ly-1..1 the row MPO is applied to env k+1 (k_mpo_apply, one workgroup per
// column) and the product is compressed back to bond D by a left-to-right
// Householder QR sweep and a right-to-left one-sided Jacobi SVD sweep
// (k_truncate_row, one workgroup walking the columns).  Everything is fp64.
//
// Layouts (D = bond cap, all row-major):
//   env  [k][c][a][u][b]  D x 2 x D box per (k,c), zero padded
//   dims [k][c]           left bond of column c of env k, c = 0..Lx
//   xbox [c][i][u][j]     2D x 2 x 2D box per column: the MPO-MPS product
//                         X_c[(a,l), u, (b,x)] and its canonical forms
#include "common.hpp"

#include <chrono>
#include <cmath>
#include <vector>

namespace {

__global__ void k_fill_dims(int *dims, int n, int v) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
        dims[t] = v;
}

// use(t, load(t)) for t = threadIdx.x, threadIdx.x + blockDim.x, ... < n, in
// that order, with the loads of SB consecutive iterations issued before any
// of their uses.  A strided loop that stores what it loads cannot move its
// next load ahead of the store (the two may alias), so it would wait out
// every load in turn.
template <int SB, class Load, class Use>
__device__ __forceinline__ void batched_loop(int n, Load &&load, Use &&use) {
    const int step = (int)blockDim.x;
    for (int t0 = threadIdx.x; t0 < n; t0 += SB * step) {
        double v[SB];
#pragma unroll
        for (int i = 0; i < SB; ++i) v[i] = t0 + i * step < n ? load(t0 + i * step) : 0.0;
#pragma unroll
        for (int i = 0; i < SB; ++i)
            if (t0 + i * step < n) use(t0 + i * step, v[i]);
    }
}

// X_c = sum_d env_{k+1,c}[a,d,b] M_{k,c}[l,u,d,x],  M = sum_s of the site
// tensor of App. A Eq. (tensor-general) with the field factor exp(beta h s);
// every column of row k, by the whole workgroup.
__device__ void mpo_apply_row(const tn_env_desc &dsc, int k) {
    __shared__ double M[2][2][2][2];   // [l][u][d][x]
    const int Lx = dsc.Lx, Ly = dsc.Ly, D = dsc.D;
    const double beta = dsc.beta;
    const double *Jh = dsc.Jh, *Jv = dsc.Jv, *h = dsc.h;
    for (int c = 0; c < Lx; ++c) {
        const int lw = c > 0 ? 2 : 1, xw = c < Lx - 1 ? 2 : 1, dw = k < Ly - 1 ? 2 : 1;
        const bool triv = (k == Ly - 1);
        const int Dl = triv ? 1 : dsc.dims[(k + 1) * (Lx + 1) + c];
        const int Dr = triv ? 1 : dsc.dims[(k + 1) * (Lx + 1) + c + 1];
        if (threadIdx.x < 16) {
            const int l = (threadIdx.x >> 3) & 1, u = (threadIdx.x >> 2) & 1;
            const int d = (threadIdx.x >> 1) & 1, x = threadIdx.x & 1;
            double acc = 0.0;
            if (l < lw && d < dw && x < xw) {
                const double hv = h ? h[k * Lx + c] : 0.0;
                for (int s = 0; s < 2; ++s) {
                    const double f = exp(beta * hv * (s ? -1.0 : 1.0));
                    const double ql = c > 0 ? tn_qleg(beta * Jh[k * (Lx - 1) + c - 1], l, s) : 1.0;
                    const double pr = c < Lx - 1 ? tn_pleg(beta * Jh[k * (Lx - 1) + c], s, x) : 1.0;
                    const double qu = tn_qleg(beta * Jv[(k - 1) * Lx + c], u, s);
                    const double pd = k < Ly - 1 ? tn_pleg(beta * Jv[k * Lx + c], s, d) : 1.0;
                    acc += f * ql * pr * qu * pd;
                }
            }
            M[l][u][d][x] = acc;
        }
        __syncthreads();
        double *X = dsc.xbox + (size_t)c * 8 * D * D;
        const int m = Dl * lw, n = Dr * xw, ld = 2 * D;
        const double *E = dsc.env + ((size_t)(k + 1) * Lx + c) * 2 * D * D;
        // the env entries of four outputs are loaded before any is stored (a
        // store to X may alias a later load of E, so the loop would otherwise
        // wait out each load in turn); the sums are those of the plain loop
        constexpr int SB = 4;
        const int nout = m * 2 * n, step = (int)blockDim.x;
        for (int t0 = threadIdx.x; t0 < nout; t0 += SB * step) {
            double ev[SB][2];
#pragma unroll
            for (int q = 0; q < SB; ++q) {
                const int t = t0 + q * step;
                const int j = t % n, a = (t / n >> 1) / lw, b = j / xw;
#pragma unroll
                for (int d = 0; d < 2; ++d)
                    ev[q][d] = (t >= nout || d >= dw) ? 0.0 : (triv ? 1.0 : E[a * 2 * D + d * D + b]);
            }
#pragma unroll
            for (int q = 0; q < SB; ++q) {
                const int t = t0 + q * step;
                if (t >= nout) break;
                const int j = t % n, rest = t / n, u = rest & 1, i = rest >> 1;
                const int l = i % lw, x = j % xw;
                double acc = 0.0;
                for (int d = 0; d < dw; ++d) acc += ev[q][d] * M[l][u][d][x];
                X[(i * 2 + u) * ld + j] = acc;
            }
        }
        if (threadIdx.x == 0) {
            dsc.xdims[c] = m;
            dsc.xdims[Lx + 1 + c] = n;
        }
        __syncthreads();
    }
}

// The factorisations below split the workgroup into rows of 16 lanes: one
// row of lanes per trailing column (QR) or per row pair (Jacobi), with
// 16-lane reductions on the VALU, so that the four 16-lane rows of a
// wavefront share every instruction.
#define TN_QW (threadIdx.x >> 4)          // 16-lane row index within the workgroup
#define TN_QL (threadIdx.x & 15)          // lane within the row
#define TN_NQW ((int)(blockDim.x >> 4))

// Column storage of the QR work matrices: LDS (D <= 32), or global memory
// read through a buffer resource, so that a lane's element addresses are
// 32-bit offsets from one scalar base (64-bit addresses per element would
// not fit the registers of the 1024-thread kernel).
template <bool GLB>
struct ColMem;
template <>
struct ColMem<false> {
    double *p;
    __device__ ColMem(double *base, uint32_t) : p(base) {}
    __device__ double ld(uint32_t idx) const { return p[idx]; }
    __device__ void st(uint32_t idx, double v) const { p[idx] = v; }
};
template <>
struct ColMem<true> {
    __amdgpu_buffer_rsrc_t rs;
    __device__ ColMem(double *base, uint32_t bytes) {
        const uint64_t a = (uint64_t)base;
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
        rs = __builtin_amdgcn_make_buffer_rsrc((void *)(((uint64_t)hi << 32) | lo), 0,
                                               (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
    }
    __device__ double ld(uint32_t idx) const {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, idx * 8u, 0, 0));
    }
    __device__ void st(uint32_t idx, double v) const {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, idx * 8u, 0, 0);
    }
};

// Elements i = j + lane + 16 e (e0 <= e < e0 + N) of the column starting at
// element c0 (m entries), one register each; entries at or beyond m read as
// zero.  The index is clamped into the column so that all N loads issue
// together (a loop bounded by m would wait for each load in turn).
template <int N, bool GLB>
__device__ __forceinline__ void col_load(const ColMem<GLB> &M, uint32_t c0, int j, int m, int e0, double (&x)[N]) {
#pragma unroll
    for (int e = 0; e < N; ++e) {
        const int i = j + TN_QL + 16 * (e0 + e);
        const double t = M.ld(c0 + (uint32_t)min(i, m - 1));
        x[e] = i < m ? t : 0.0;
    }
}

// col <- col - t (v . col) v over rows j .. m-1 of the column starting at
// element c, with v the reflector stored in the column starting at vc below
// row j and an implicit 1 at row j.  Columns of up to 128 rows (MPL <= 8)
// keep v in registers across the columns a lane row updates (vreg, loaded
// by the caller); longer ones read v and the column in chunks of eight,
// twice (for the product and for the update), to bound the registers.
template <int MPL, bool GLB>
__device__ __forceinline__ void reflect_col(const ColMem<GLB> &M, uint32_t c, uint32_t vc,
                                            const double (&vreg)[MPL < 8 ? MPL : 8], int j, int m, double t) {
    constexpr int CH = MPL < 8 ? MPL : 8;
    static_assert(MPL % CH == 0, "whole chunks");
    double dot = 0.0;
    if constexpr (MPL == CH) {
        double y[CH];
        col_load<CH, GLB>(M, c, j, m, 0, y);
#pragma unroll
        for (int e = 0; e < CH; ++e) dot += vreg[e] * y[e];
        dot = tn_row16_sum(dot) * t;
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int i = j + TN_QL + 16 * e;
            if (i < m) M.st(c + i, y[e] - dot * vreg[e]);
        }
    } else {
        auto vchunk = [&](int e0, double (&v)[CH]) {
            col_load<CH, GLB>(M, vc, j, m, e0, v);
            if (e0 == 0 && TN_QL == 0) v[0] = 1.0;
        };
#pragma unroll
        for (int e0 = 0; e0 < MPL; e0 += CH) {
            double v[CH], y[CH];
            vchunk(e0, v);
            col_load<CH, GLB>(M, c, j, m, e0, y);
#pragma unroll
            for (int e = 0; e < CH; ++e) dot += v[e] * y[e];
        }
        dot = tn_row16_sum(dot) * t;
#pragma unroll
        for (int e0 = 0; e0 < MPL; e0 += CH) {
            double v[CH], y[CH];
            vchunk(e0, v);
            col_load<CH, GLB>(M, c, j, m, e0, y);
#pragma unroll
            for (int e = 0; e < CH; ++e) {
                const int i = j + TN_QL + 16 * (e0 + e);
                if (i < m) M.st(c + i, y[e] - dot * v[e]);
            }
        }
    }
}

// The reflector's elements per lane, its leading 1 included, for reflect_col
// (columns of up to 128 rows only).
template <int MPL, bool GLB>
__device__ __forceinline__ void reflector_regs(const ColMem<GLB> &M, uint32_t vc, int j, int m,
                                               double (&v)[MPL < 8 ? MPL : 8]) {
    if constexpr (MPL <= 8) {
        col_load<MPL, GLB>(M, vc, j, m, 0, v);
        if (TN_QL == 0) v[0] = 1.0;
    }
}

// Householder QR of A (m x n, column-major, A[j*lda + i] = A(i, j); m <= 16
// MPL): R in the upper triangle, reflector j = (1, A(j+1:, j)) with
// coefficient tau[j].  Column-major storage keeps the 16 lanes of a row on
// consecutive words.
template <int MPL, bool GLB>
__device__ void qw_householder(double *A, int m, int n, int lda, double *tau) {
    const ColMem<GLB> M(A, (uint32_t)((size_t)lda * n * sizeof(double)));
    constexpr int CH = MPL < 8 ? MPL : 8;
    const int kk = min(m, n);
    for (int j = 0; j < kk; ++j) {
        const uint32_t cj = (uint32_t)j * lda;
        if (TN_QW == 0) {
            double s2 = 0.0;
#pragma unroll
            for (int e0 = 0; e0 < MPL; e0 += CH) {
                double x[CH];
                col_load<CH, GLB>(M, cj, j + 1, m, e0, x);
#pragma unroll
                for (int e = 0; e < CH; ++e) s2 += x[e] * x[e];
            }
            s2 = tn_row16_sum(s2);
            const double alpha = M.ld(cj + j);
            double t = 0.0, scl = 0.0, beta = alpha;
            if (s2 > 0.0) {
                beta = -copysign(sqrt(alpha * alpha + s2), alpha);
                t = (beta - alpha) / beta;
                scl = 1.0 / (alpha - beta);
            }
#pragma unroll
            for (int e0 = 0; e0 < MPL; e0 += CH) {
                double x[CH];
                col_load<CH, GLB>(M, cj, j + 1, m, e0, x);
#pragma unroll
                for (int e = 0; e < CH; ++e) {
                    const int i = j + 1 + TN_QL + 16 * (e0 + e);
                    if (i < m) M.st(cj + i, x[e] * scl);
                }
            }
            if (TN_QL == 0) {
                M.st(cj + j, beta);
                tau[j] = t;
            }
        }
        __syncthreads();
        const double t = tau[j];
        if (t != 0.0) {
            double v[CH];
            reflector_regs<MPL, GLB>(M, cj, j, m, v);
            for (int l = j + 1 + TN_QW; l < n; l += TN_NQW)
                reflect_col<MPL, GLB>(M, (uint32_t)l * lda, cj, v, j, m, t);
        }
        __syncthreads();
    }
}

// Q (m x kk, column-major, ld ldq) = H_0 ... H_{kk-1} [I; 0] from the
// reflectors in A (as left by qw_householder).
template <int MPL, bool GLB>
__device__ void qw_form_q(double *A, int m, int n, int lda, const double *tau, double *Q, int ldq) {
    const int kk = min(m, n);
    const ColMem<GLB> MA(A, (uint32_t)((size_t)lda * n * sizeof(double)));
    const ColMem<GLB> MQ(Q, (uint32_t)((size_t)ldq * kk * sizeof(double)));
    constexpr int CH = MPL < 8 ? MPL : 8;
    for (int t = threadIdx.x; t < m * kk; t += blockDim.x) {
        const int l = t / m, i = t % m;
        Q[(size_t)l * ldq + i] = (i == l) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = kk - 1; j >= 0; --j) {
        const double tj = tau[j];
        const uint32_t cj = (uint32_t)j * lda;
        if (tj != 0.0) {
            double v[CH];
            reflector_regs<MPL, GLB>(MA, cj, j, m, v);
            for (int l = j + TN_QW; l < kk; l += TN_NQW) {
                if constexpr (MPL <= 8) {
                    reflect_col<MPL, GLB>(MQ, (uint32_t)l * ldq, 0, v, j, m, tj);
                } else {
                    // the reflector lives in A, the column in Q: read both by chunks
                    double dot = 0.0;
#pragma unroll
                    for (int e0 = 0; e0 < MPL; e0 += CH) {
                        double w[CH], y[CH];
                        col_load<CH, GLB>(MA, cj, j, m, e0, w);
                        if (e0 == 0 && TN_QL == 0) w[0] = 1.0;
                        col_load<CH, GLB>(MQ, (uint32_t)l * ldq, j, m, e0, y);
#pragma unroll
                        for (int e = 0; e < CH; ++e) dot += w[e] * y[e];
                    }
                    dot = tn_row16_sum(dot) * tj;
#pragma unroll
                    for (int e0 = 0; e0 < MPL; e0 += CH) {
                        double w[CH], y[CH];
                        col_load<CH, GLB>(MA, cj, j, m, e0, w);
                        if (e0 == 0 && TN_QL == 0) w[0] = 1.0;
                        col_load<CH, GLB>(MQ, (uint32_t)l * ldq, j, m, e0, y);
#pragma unroll
                        for (int e = 0; e < CH; ++e) {
                            const int i = j + TN_QL + 16 * (e0 + e);
                            if (i < m) MQ.st((uint32_t)l * ldq + i, y[e] - dot * w[e]);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

// One-sided (Hestenes) Jacobi on the rows of W [n][len] (ld ldw, len <= 128,
// rows zero padded to 16 NQ entries): plane rotations of row pairs in the
// parallel round-robin order, until every pair is orthogonal to relative
// tolerance 4*len*eps, or a sweep rotated no pair by more than a tangent of
// 1e-8.  Rows whose squared norm is below small2 =
// (len*eps)^2 ||W||_F^2 are numerically zero and not rotated.  The squared
// row norms are recomputed at the start of every sweep and updated exactly by
// each rotation (a - t g, b + t g), so a pair needs only its inner product.
// NQ, the 16-wide slices of a row, is fixed at compile time so that a lane's
// entries load together.  Returns the number of sweeps, or -1 without
// convergence.
template <int NQ>
__device__ int qw_jacobi_nq(double *W, int n, int len, int ldw, double small2, double *nrm,
                            int *flag) {
    if (n <= 1) return 0;
    const int npad = n + (n & 1), nr = npad - 1;
    const double tol = 4.0 * len * 2.220446049250313e-16;
    const double tol2 = tol * tol;
    for (int sweep = 0; sweep < 60; ++sweep) {
        for (int i = TN_QW; i < n; i += TN_NQW) {
            double v[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) v[q] = W[i * ldw + TN_QL + 16 * q];
            double s2 = 0.0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) s2 += v[q] * v[q];
            s2 = tn_row16_sum(s2);
            if (TN_QL == 0) nrm[i] = s2;
        }
        if (threadIdx.x == 0) *flag = 0;
        __syncthreads();
        for (int t = 0; t < nr; ++t) {
            for (int p = TN_QW; p < npad / 2; p += TN_NQW) {
                int i, j;
                if (p == 0) {
                    i = nr;
                    j = t;
                } else {
                    i = t + p;
                    if (i >= nr) i -= nr;
                    j = t - p;
                    if (j < 0) j += nr;
                }
                if (i >= n || j >= n) continue;
                const double a = nrm[i], b = nrm[j];   // read with the rows, ahead of the reduction
                double x[NQ], y[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    x[q] = W[i * ldw + TN_QL + 16 * q];
                    y[q] = W[j * ldw + TN_QL + 16 * q];
                }
                double g = 0.0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) g += x[q] * y[q];
                g = tn_row16_sum(g);
                if (a > small2 && b > small2 && g * g > tol2 * a * b) {
                    // t = tan of the angle that makes the pair orthogonal.  Only
                    // the rotation's orthogonality must be exact (cs = (1 +
                    // t^2)^-1/2 to rounding, sn = cs t); an angle a few ulps
                    // off leaves a residual inner product of that relative
                    // size, which later rotations remove.  So the square root
                    // and the reciprocal in t use the hardware estimates with
                    // one Newton step each.
                    const double d = b - a;
                    const double qq = d * d + 4.0 * g * g;   // > 0: g != 0 here
                    double rq = __builtin_amdgcn_rsq(qq);
                    rq = rq * fma(-0.5 * qq * rq, rq, 1.5);
                    const double den = fabs(d) + qq * rq;
                    double rd = __builtin_amdgcn_rcp(den);
                    rd = rd * fma(-den, rd, 2.0);
                    const double tt = (d < 0.0 ? -2.0 * g : 2.0 * g) * rd;
                    const double cs = rsqrt(1.0 + tt * tt), sn = cs * tt;
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        W[i * ldw + TN_QL + 16 * q] = cs * x[q] - sn * y[q];
                        W[j * ldw + TN_QL + 16 * q] = sn * x[q] + cs * y[q];
                    }
                    if (TN_QL == 0) {
                        nrm[i] = fmax(a - tt * g, 0.0);
                        nrm[j] = b + tt * g;
                        // a sweep whose rotations all have |t| <= 1e-8 leaves
                        // inner products of order t^2 ~ 1e-16 relative (the
                        // convergence of cyclic Jacobi is quadratic): no
                        // further sweep is needed to confirm
                        if (fabs(tt) > 1e-8) *flag = 1;
                    }
                }
            }
            __syncthreads();
        }
        const int any = *flag;
        __syncthreads();
        if (!any) return sweep;
    }
    return -1;
}

// len <= 16 SL (SL: the largest count of 16-wide slices of a row)
template <int SL>
__device__ int qw_jacobi(double *W, int n, int len, int ldw, double small2, double *nrm, int *flag) {
    switch (min((len + 15) >> 4, SL)) {   // 16-wide slices per row (rows are zero padded to them)
    case 1: return qw_jacobi_nq<1>(W, n, len, ldw, small2, nrm, flag);
    case 2: return qw_jacobi_nq<2>(W, n, len, ldw, small2, nrm, flag);
    case 3: return qw_jacobi_nq<3>(W, n, len, ldw, small2, nrm, flag);
    case 4: return qw_jacobi_nq<4>(W, n, len, ldw, small2, nrm, flag);
    }
    if constexpr (SL > 4) {
        switch ((len + 15) >> 4) {
        case 5: return qw_jacobi_nq<5>(W, n, len, ldw, small2, nrm, flag);
        case 6: return qw_jacobi_nq<6>(W, n, len, ldw, small2, nrm, flag);
        case 7: return qw_jacobi_nq<7>(W, n, len, ldw, small2, nrm, flag);
        default: return qw_jacobi_nq<8>(W, n, len, ldw, small2, nrm, flag);
        }
    }
    return -1;
}

// Doubles of the SVD matrix (2D rows, zero padded to 16-wide slices, odd
// leading dimension) and of one work area (an 4D x 2D matrix with an odd
// leading dimension, or the SVD matrix and its copy).
__host__ __device__ constexpr size_t tn_svd_area(int D) {
    return (size_t)2 * D * ((((size_t)2 * D + 15) & ~(size_t)15) + 1);
}
__host__ __device__ constexpr size_t tn_qr_area(int D) {
    return (size_t)8 * D * D + 4 * D > 2 * tn_svd_area(D) ? (size_t)8 * D * D + 4 * D
                                                            : 2 * tn_svd_area(D);
}

// Scratch of the two-site variational sweeps, in doubles: [0] ln of the norm
// the QR sweep removed; xh the normalised product X^ (left-canonical boxes of
// xbox); ps the fitted MPS psi (same boxes); re / ls the right / left
// overlaps of psi with X^ per column ([chi][A], row stride 2 D); t1, t2, th
// the intermediate products of one two-site tensor.
struct FitLayout {
    size_t xh, ps, re, ls, t1, t2, th, total;
};
__host__ __device__ inline FitLayout fit_layout(int Lx, int D) {
    const size_t box = (size_t)8 * D * D, m2 = (size_t)2 * D * D;
    FitLayout f;
    size_t o = 8;
    f.xh = o;
    o += (size_t)Lx * box;
    f.ps = o;
    o += (size_t)Lx * box;
    f.re = o;
    o += (size_t)(Lx + 1) * m2;
    f.ls = o;
    o += (size_t)(Lx + 1) * m2;
    f.t1 = o;
    o += (size_t)4 * D * D;
    f.t2 = o;
    o += (size_t)8 * D * D;
    f.th = o;
    o += (size_t)4 * D * D;
    f.total = o;
    return f;
}
// the bond dimensions of X^ are kept in xdims from this offset (ints)
constexpr int FIT_DIMS = 1024;

// Compress the MPO-MPS product of row k held in xbox and store env k.
// Work areas (doubles): QA [8 D^2 + 4 D] the QR matrix, later the SVD matrix
// W and a copy of it; QB (same size) Q, then the staged right neighbour,
// later Z = U S and Y = X_{c-1} Z.  QLDS: QA and QB in LDS (D <= 32);
// otherwise they are in global `gwork` and only W sits in LDS.
template <bool QLDS>
__device__ void truncate_row(const tn_env_desc &dsc, int k, double *lds, double lognorm0) {
    const int Lx = dsc.Lx, D = dsc.D;
    double *xbox = dsc.xbox, *env = dsc.env, *ell = dsc.ell, *gwork = dsc.wbuf;
    int *xdims = dsc.xdims, *dims = dsc.dims, *cst = dsc.cst;
    unsigned long long *counters = dsc.counters;
    __shared__ double tau[2 * TN_MAX_D];
    __shared__ double sv[2 * TN_MAX_D];
    __shared__ double nrm[2 * TN_MAX_D];
    __shared__ int idx[2 * TN_MAX_D];
    __shared__ int mX[4 * TN_MAX_D + 1], nX[4 * TN_MAX_D + 1];
    __shared__ double red[16];
    __shared__ int flag;
    __shared__ int cmin;
    if (threadIdx.x == 0) cmin = -1;

    const size_t D2 = (size_t)D * D;
    const size_t SZ = tn_qr_area(D);       // one work area, padded leading dimensions
    double *QA = QLDS ? lds : gwork;
    double *QB = QA + SZ;
    double *W = lds;                       // SVD matrix (aliases QA when QLDS)
    double *Worig = QA + tn_svd_area(D);   // its unrotated copy
    double *Z = QB, *Y = QB + 2 * D2;
    const int ld = 2 * D;
    const size_t box = (size_t)8 * D2;
    const double eps = 2.220446049250313e-16;
    constexpr int QSB = QLDS ? 8 : 4;   // loads batched per staging loop (registers)

    for (int c = threadIdx.x; c < Lx; c += blockDim.x) {
        mX[c] = xdims[c];
        nX[c] = xdims[Lx + 1 + c];
    }
    __syncthreads();

    // ---- left-to-right QR sweep: X_c <- Q, X_{c+1} <- R X_{c+1} / |X_c|.
    // The carried factor is kept at unit norm and its norm logged: a row's
    // weight can pass the fp64 range before the sweep ends.
    double lognorm = lognorm0;
    for (int c = 0; c + 1 < Lx; ++c) {
        double *X = xbox + c * box, *Xn = xbox + (c + 1) * box;
        const int m = 2 * mX[c], n = nX[c], n1 = nX[c + 1];
        const int lda = m | 1;   // odd leading dimension: lanes of a row on distinct banks
        double x2 = 0.0;
        batched_loop<QSB>(m * n, [&](int t) { return X[(t / n) * ld + t % n]; }, [&](int t, double v) {
            QA[(size_t)(t % n) * lda + t / n] = v;
            x2 += v * v;
        });
        x2 = tn_block_sum(x2, red);   // ends with a barrier: QA is complete
        const double xn = sqrt(x2);
        const double xinv = xn > 0.0 ? 1.0 / xn : 1.0;
        if (xn > 0.0) lognorm += log(xn);
        qw_householder<QLDS ? 8 : 16, !QLDS>(QA, m, n, lda, tau);   // m <= 4 D
        const int kk = min(m, n);
        qw_form_q<QLDS ? 8 : 16, !QLDS>(QA, m, n, lda, tau, QB, lda);
        for (int t = threadIdx.x; t < m * kk; t += blockDim.x) {
            const int r = t / kk, l = t % kk;
            X[r * ld + l] = QB[(size_t)l * lda + r];
        }
        __syncthreads();
        // stage X_{c+1} [q][(u, j)] (n rows), then T = R X_{c+1} into its first kk rows
        const int w1 = 2 * n1;
        batched_loop<QSB>(n * w1, [&](int t) {
            const int q = t / w1, e = t % w1;
            return Xn[(q * 2 + e / n1) * ld + e % n1];
        }, [&](int t, double v) { QB[t] = v; });
        __syncthreads();
        for (int t = threadIdx.x; t < kk * w1; t += blockDim.x) {
            const int p = t / w1, e = t % w1;
            double acc = 0.0;
            for (int q = p; q < n; ++q) acc += QA[(size_t)q * lda + p] * QB[q * w1 + e];
            Xn[(p * 2 + e / n1) * ld + e % n1] = acc * xinv;
        }
        if (threadIdx.x == 0) {
            mX[c + 1] = kk;
            nX[c] = kk;
        }
        __syncthreads();
    }

    // ---- normalise the last column (with the logged factors, its norm is
    // the norm of the state)
    {
        double *X = xbox + (Lx - 1) * box;
        const int m = mX[Lx - 1], n = nX[Lx - 1];
        double s2 = 0.0;
        for (int t = threadIdx.x; t < m * 2 * n; t += blockDim.x) {
            const int r = t / n, j = t % n;
            s2 += X[r * ld + j] * X[r * ld + j];
        }
        s2 = tn_block_sum(s2, red);
        const double nrm = sqrt(s2);
        const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
        for (int t = threadIdx.x; t < m * 2 * n; t += blockDim.x) {
            const int r = t / n, j = t % n;
            X[r * ld + j] *= inv;
        }
        lognorm += log(nrm);
        __syncthreads();
    }
    if (dsc.fit > 0) {   // keep the normalised product for the variational sweeps
        const FitLayout F = fit_layout(Lx, D);
        for (size_t t = threadIdx.x; t < (size_t)Lx * box; t += blockDim.x) dsc.fbuf[F.xh + t] = xbox[t];
        for (int c = threadIdx.x; c <= Lx; c += blockDim.x) xdims[FIT_DIMS + c] = c < Lx ? mX[c] : nX[Lx - 1];
        if (threadIdx.x == 0) dsc.fbuf[0] = lognorm;
        __syncthreads();
    }

    // ---- right-to-left SVD sweep with truncation to D
    for (int c = Lx - 1; c >= 1; --c) {
        double *X = xbox + c * box, *Xp = xbox + (c - 1) * box;
        const int rows = mX[c], ncol = nX[c], len = 2 * ncol;
        const int lenp = (len + 15) & ~15;   // zero padded to 16-wide slices
        const int ldw = lenp | 1;            // odd: rows of W on distinct banks
        double f2 = 0.0;
        batched_loop<QSB>(rows * lenp, [&](int t) {
            const int i = t / lenp, e = t % lenp;
            return e < len ? X[(i * 2 + e / ncol) * ld + e % ncol] : 0.0;
        }, [&](int t, double v) {
            const int i = t / lenp, e = t % lenp;
            W[i * ldw + e] = v;
            Worig[i * ldw + e] = v;
            f2 += v * v;
        });
        f2 = tn_block_sum(f2, red);
        const double zero2 = f2 * (len * eps) * (len * eps);
        const int sweeps = qw_jacobi<QLDS ? 4 : 8>(W, rows, len, ldw, zero2, nrm, &flag);   // len <= 2 D
        if (sweeps < 0 && threadIdx.x == 0) atomicAdd(&counters[CNT_NOCONV], 1ull);
        for (int i = TN_QW; i < rows; i += TN_NQW) {
            double s2 = 0.0;
            for (int e = TN_QL; e < lenp; e += 16) s2 += W[i * ldw + e] * W[i * ldw + e];
            s2 = tn_row16_sum(s2);
            if (TN_QL == 0) sv[i] = s2 > zero2 ? sqrt(s2) : 0.0;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < rows; i += blockDim.x) {
            int r = 0;
            const double si = sv[i];
            for (int j = 0; j < rows; ++j) r += (sv[j] > si) || (sv[j] == si && j < i);
            idx[r] = i;
        }
        __syncthreads();
        const int nsv = min(rows, len);
        const int chi = min(D, nsv);
        if (threadIdx.x == 0 && chi < nsv) {
            cmin = c;   // the sweep runs right to left: the last cut is the leftmost
            if (sv[idx[chi - 1]] - sv[idx[chi]] < 1e-12 * sv[idx[0]])
                atomicAdd(&counters[CNT_DEGEN], 1ull);
        }
        // Z = U[:, :chi] S[:chi] = Worig W'[idx]^T / s  (the rotated rows are S V^T);
        // consecutive threads take consecutive rows r of Worig for one kept row
        for (int t = threadIdx.x; t < rows * chi; t += blockDim.x) {
            const int kq = t / rows, r = t % rows, ik = idx[kq];
            const double s = sv[ik];
            double acc = 0.0;
            if (s > 0.0) {
                for (int e = 0; e < len; ++e) acc += Worig[r * ldw + e] * W[ik * ldw + e];
                acc /= s;
            }
            Z[r * chi + kq] = acc;
        }
        __syncthreads();
        // Y = X_{c-1} Z, X_c <- V^T[:chi]
        const int m1 = 2 * mX[c - 1];
        for (int t = threadIdx.x; t < m1 * chi; t += blockDim.x) {
            const int r = t / chi, kq = t % chi;
            // the same sum in the same order, QSB loads of X at a time
            const double *xr = Xp + r * ld;
            double acc = 0.0;
            int q = 0;
            for (; q + QSB <= rows; q += QSB) {
                double xv[QSB];
#pragma unroll
                for (int i = 0; i < QSB; ++i) xv[i] = xr[q + i];
#pragma unroll
                for (int i = 0; i < QSB; ++i) acc += xv[i] * Z[(q + i) * chi + kq];
            }
            for (; q < rows; ++q) acc += xr[q] * Z[q * chi + kq];
            Y[t] = acc;
        }
        for (int t = threadIdx.x; t < chi * len; t += blockDim.x) {
            const int kq = t / len, e = t % len;
            const int ik = idx[kq];
            const double s = sv[ik];
            X[(kq * 2 + e / ncol) * ld + e % ncol] = s > 0.0 ? W[ik * ldw + e] / s : 0.0;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < m1 * chi; t += blockDim.x) Xp[(t / chi) * ld + t % chi] = Y[t];
        if (threadIdx.x == 0) {
            mX[c] = chi;
            nX[c - 1] = chi;
        }
        __syncthreads();
    }

    // ---- normalise column 0 and store env k
    {
        double *X = xbox;
        const int m = mX[0], n = nX[0];
        double s2 = 0.0;
        for (int t = threadIdx.x; t < m * 2 * n; t += blockDim.x) {
            const int r = t / n, j = t % n;
            s2 += X[r * ld + j] * X[r * ld + j];
        }
        s2 = tn_block_sum(s2, red);
        const double nrm = sqrt(s2);
        const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
        for (int t = threadIdx.x; t < m * 2 * n; t += blockDim.x) {
            const int r = t / n, j = t % n;
            X[r * ld + j] *= inv;
        }
        lognorm += log(nrm);
        __syncthreads();
    }
    for (size_t t = threadIdx.x; t < (size_t)Lx * 2 * D * D; t += blockDim.x) {
        const int c = (int)(t / (2 * D * D));
        const int rem = (int)(t % (2 * D * D));
        const int a = rem / (2 * D), u = (rem / D) & 1, b = rem % D;
        double v = 0.0;
        if (a < mX[c] && b < nX[c]) v = xbox[c * box + (a * 2 + u) * ld + b];
        env[((size_t)k * Lx) * 2 * D * D + t] = v;
    }
    for (int c = threadIdx.x; c <= Lx; c += blockDim.x)
        dims[k * (Lx + 1) + c] = c < Lx ? mX[c] : 1;
    if (threadIdx.x == 0) {
        ell[k] = lognorm;
        cst[k] = cmin;
    }
    __syncthreads();
}

// ---- two-site variational sweeps (run after truncate_row stored env k) ----
// Bond dimensions: hd[c] of X^ (left bond of column c, c = 0..Lx), pd[c] of
// psi.  Boxes of X^ and psi: [(A * 2 + u) * 2D + B] per column, as xbox.

// Theta of bond (c, c+1) as a [(a u)][(v b)] matrix in th:
//   Theta = sum L[a][A] X^_c[A][u][M] X^_{c+1}[M][v][B] R[b][B]
// with the left overlap L ([ca][A0]) and the right overlap R ([cb][A2]).
__device__ void fit_theta(const double *XH, const double *Lm, const double *Rm, double *t1, double *t2,
                          double *th, int c, int ca, int cb, int A0, int A1, int A2, int D) {
    const int ld = 2 * D;
    const size_t box = (size_t)8 * D * D;
    const double *X0 = XH + (size_t)c * box, *X1 = XH + (size_t)(c + 1) * box;
    for (int t = threadIdx.x; t < ca * 2 * A1; t += blockDim.x) {
        const int r = t / A1, M = t % A1, a = r >> 1, u = r & 1;
        double acc = 0.0;
        for (int A = 0; A < A0; ++A) acc += Lm[a * ld + A] * X0[(A * 2 + u) * ld + M];
        t1[t] = acc;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ca * 2 * 2 * A2; t += blockDim.x) {
        const int r = t / (2 * A2), e = t % (2 * A2), v = e / A2, B = e % A2;
        double acc = 0.0;
        for (int M = 0; M < A1; ++M) acc += t1[r * A1 + M] * X1[(M * 2 + v) * ld + B];
        t2[t] = acc;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ca * 2 * 2 * cb; t += blockDim.x) {
        const int r = t / (2 * cb), e = t % (2 * cb), v = e / cb, b = e % cb;
        double acc = 0.0;
        for (int B = 0; B < A2; ++B) acc += t2[(r * 2 + v) * A2 + B] * Rm[b * ld + B];
        th[t] = acc;
    }
    __syncthreads();
}

// SVD of Theta truncated to D by one-sided Jacobi on the rows of W.  A
// left-to-right step (lr) takes W = Theta^T, so the rotated rows give U:
// psi_c = U (left-canonical), psi_{c+1} = S V^T = (Theta^T U)^T.  A right-to-
// left step takes W = Theta: psi_{c+1} = V^T (right-canonical),
// psi_c = U S = Theta V.  Returns the kept bond dimension.
__device__ int fit_split(const double *th, int ca, int cb, bool lr, double *W, double *Wo, int D, double *sv,
                         double *nrm, int *idx, int *flag, double *red, unsigned long long *counters,
                         double *Pc, double *Pc1) {
    const int ld = 2 * D;
    const int rows = lr ? 2 * cb : 2 * ca, len = lr ? 2 * ca : 2 * cb;
    const int lenp = (len + 15) & ~15, ldw = lenp | 1;
    const double eps = 2.220446049250313e-16;
    double f2 = 0.0;
    for (int t = threadIdx.x; t < rows * lenp; t += blockDim.x) {
        const int i = t / lenp, e = t % lenp;
        const double v = e < len ? (lr ? th[e * (2 * cb) + i] : th[i * (2 * cb) + e]) : 0.0;
        W[i * ldw + e] = v;
        Wo[i * ldw + e] = v;
        f2 += v * v;
    }
    f2 = tn_block_sum(f2, red);
    const double zero2 = f2 * (len * eps) * (len * eps);
    const int sweeps = qw_jacobi<4>(W, rows, len, ldw, zero2, nrm, flag);   // len <= 2 D <= 64
    if (sweeps < 0 && threadIdx.x == 0) atomicAdd(&counters[CNT_NOCONV], 1ull);
    for (int i = TN_QW; i < rows; i += TN_NQW) {
        double s2 = 0.0;
        for (int e = TN_QL; e < lenp; e += 16) s2 += W[i * ldw + e] * W[i * ldw + e];
        s2 = tn_row16_sum(s2);
        if (TN_QL == 0) sv[i] = s2 > zero2 ? sqrt(s2) : 0.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < rows; i += blockDim.x) {
        int r = 0;
        const double si = sv[i];
        for (int j = 0; j < rows; ++j) r += (sv[j] > si) || (sv[j] == si && j < i);
        idx[r] = i;
    }
    __syncthreads();
    const int chi = min(D, min(rows, len));
    // a cut tied to 1e-12 of the largest singular value is counted (rounding
    // decides which vectors are kept), as in the successive-SVD sweep
    if (threadIdx.x == 0 && chi < min(rows, len) && sv[idx[chi - 1]] - sv[idx[chi]] < 1e-12 * sv[idx[0]])
        atomicAdd(&counters[CNT_DEGEN], 1ull);
    // orthonormal factor O[k][e] = W'[idx k][e] / s_k (length len); coefficients
    // C[i][k] = sum_e Wo[i][e] O[k][e] (rows x chi)
    for (int t = threadIdx.x; t < chi * len; t += blockDim.x) {
        const int kq = t / len, e = t % len, ik = idx[kq];
        const double s = sv[ik];
        const double o = s > 0.0 ? W[ik * ldw + e] / s : 0.0;
        if (lr) {   // e = (a u): psi_c[a][u][kq]
            Pc[e * ld + kq] = o;
        } else {    // e = (v b): psi_{c+1}[kq][v][b]
            const int v = e / cb, b = e % cb;
            Pc1[(kq * 2 + v) * ld + b] = o;
        }
    }
    for (int t = threadIdx.x; t < rows * chi; t += blockDim.x) {
        const int kq = t / rows, i = t % rows, ik = idx[kq];
        const double s = sv[ik];
        double acc = 0.0;
        if (s > 0.0) {
            for (int e = 0; e < len; ++e) acc += Wo[i * ldw + e] * W[ik * ldw + e];
            acc /= s;
        }
        if (lr) {   // i = (v b): psi_{c+1}[kq][v][b]
            const int v = i / cb, b = i % cb;
            Pc1[(kq * 2 + v) * ld + b] = acc;
        } else {    // i = (a u): psi_c[a][u][kq]
            Pc[i * ld + kq] = acc;
        }
    }
    __syncthreads();
    return chi;
}

// R_j[a][A] = sum_{u, b, B} psi_j[a][u][b] X^_j[A][u][B] R_{j+1}[b][B]
__device__ void fit_right(const double *XH, const double *PS, double *RE, double *t1, const int *hd,
                          const int *pd, int j, int D) {
    const int ld = 2 * D;
    const size_t box = (size_t)8 * D * D, m2 = (size_t)2 * D * D;
    const int cj = pd[j], cn = pd[j + 1], Aj = hd[j], An = hd[j + 1];
    const double *X = XH + (size_t)j * box, *P = PS + (size_t)j * box, *Rn = RE + (size_t)(j + 1) * m2;
    double *Rj = RE + (size_t)j * m2;
    for (int t = threadIdx.x; t < Aj * 2 * cn; t += blockDim.x) {
        const int r = t / cn, b = t % cn;
        double acc = 0.0;
        for (int B = 0; B < An; ++B) acc += X[r * ld + B] * Rn[b * ld + B];
        t1[t] = acc;   // [(A u)][b]
    }
    __syncthreads();
    for (int t = threadIdx.x; t < cj * Aj; t += blockDim.x) {
        const int a = t / Aj, A = t % Aj;
        double acc = 0.0;
        for (int u = 0; u < 2; ++u)
            for (int b = 0; b < cn; ++b) acc += P[(a * 2 + u) * ld + b] * t1[(A * 2 + u) * cn + b];
        Rj[a * ld + A] = acc;
    }
    __syncthreads();
}

// L_{j+1}[k][M] = sum_{a, u, A} psi_j[a][u][k] L_j[a][A] X^_j[A][u][M]
__device__ void fit_left(const double *XH, const double *PS, double *LS, double *t1, const int *hd,
                         const int *pd, int j, int D) {
    const int ld = 2 * D;
    const size_t box = (size_t)8 * D * D, m2 = (size_t)2 * D * D;
    const int cj = pd[j], cn = pd[j + 1], Aj = hd[j], An = hd[j + 1];
    const double *X = XH + (size_t)j * box, *P = PS + (size_t)j * box, *Lj = LS + (size_t)j * m2;
    double *Ln = LS + (size_t)(j + 1) * m2;
    for (int t = threadIdx.x; t < cj * 2 * An; t += blockDim.x) {
        const int r = t / An, M = t % An, a = r >> 1, u = r & 1;
        double acc = 0.0;
        for (int A = 0; A < Aj; ++A) acc += Lj[a * ld + A] * X[(A * 2 + u) * ld + M];
        t1[t] = acc;   // [(a u)][M]
    }
    __syncthreads();
    for (int t = threadIdx.x; t < cn * An; t += blockDim.x) {
        const int kq = t / An, M = t % An;
        double acc = 0.0;
        for (int r = 0; r < 2 * cj; ++r) acc += P[r * ld + kq] * t1[r * An + M];
        Ln[kq * ld + M] = acc;
    }
    __syncthreads();
}

// The variational sweeps of row k: fit psi (starting from the stored env k
// with its norm put back) to X^, then store the normalised psi as env k with
// ell_k = ln |X| (QR sweep) + ln |psi|.
__device__ void fit_row(const tn_env_desc &dsc, int k, double *lds) {
    const int Lx = dsc.Lx, D = dsc.D, ld = 2 * D;
    const size_t box = (size_t)8 * D * D, m2 = (size_t)2 * D * D;
    const FitLayout F = fit_layout(Lx, D);
    double *fb = dsc.fbuf;
    double *XH = fb + F.xh, *PS = fb + F.ps, *RE = fb + F.re, *LS = fb + F.ls;
    double *t1 = fb + F.t1, *t2 = fb + F.t2, *th = fb + F.th;
    double *W = lds, *Wo = lds + tn_svd_area(D);
    __shared__ int hd[4 * TN_MAX_D + 1], pd[4 * TN_MAX_D + 1];
    __shared__ double sv[2 * TN_MAX_D], nrm[2 * TN_MAX_D];
    __shared__ int idx[2 * TN_MAX_D];
    __shared__ double red[16];
    __shared__ int flag;
    const double lnqr = fb[0];
    const double m0 = exp(dsc.ell[k] - lnqr);   // norm of the SVD start, <= 1
    for (int c = threadIdx.x; c <= Lx; c += blockDim.x) {
        hd[c] = dsc.xdims[FIT_DIMS + c];
        pd[c] = c < Lx ? dsc.dims[k * (Lx + 1) + c] : 1;
    }
    const double *E = dsc.env + (size_t)k * Lx * 2 * D * D;
    for (size_t t = threadIdx.x; t < (size_t)Lx * 2 * D * D; t += blockDim.x) {
        const int c = (int)(t / (2 * D * D));
        const int rem = (int)(t % (2 * D * D));
        const int a = rem / (2 * D), u = (rem / D) & 1, b = rem % D;
        PS[c * box + (a * 2 + u) * ld + b] = c == 0 ? E[t] * m0 : E[t];
    }
    if (threadIdx.x == 0) {
        LS[0] = 1.0;
        RE[(size_t)Lx * m2] = 1.0;
    }
    __syncthreads();
    if (Lx > 1) {
        for (int j = Lx - 1; j >= 2; --j) fit_right(XH, PS, RE, t1, hd, pd, j, D);
        for (int sweep = 0; sweep < dsc.fit; ++sweep) {
            for (int c = 0; c + 1 < Lx; ++c) {   // left to right
                fit_theta(XH, LS + (size_t)c * m2, RE + (size_t)(c + 2) * m2, t1, t2, th, c, pd[c], pd[c + 2],
                          hd[c], hd[c + 1], hd[c + 2], D);
                const int chi = fit_split(th, pd[c], pd[c + 2], true, W, Wo, D, sv, nrm, idx, &flag, red,
                                          dsc.counters, PS + (size_t)c * box, PS + (size_t)(c + 1) * box);
                if (threadIdx.x == 0) pd[c + 1] = chi;
                __syncthreads();
                fit_left(XH, PS, LS, t1, hd, pd, c, D);
            }
            for (int c = Lx - 2; c >= 0; --c) {   // right to left
                fit_theta(XH, LS + (size_t)c * m2, RE + (size_t)(c + 2) * m2, t1, t2, th, c, pd[c], pd[c + 2],
                          hd[c], hd[c + 1], hd[c + 2], D);
                const int chi = fit_split(th, pd[c], pd[c + 2], false, W, Wo, D, sv, nrm, idx, &flag, red,
                                          dsc.counters, PS + (size_t)c * box, PS + (size_t)(c + 1) * box);
                if (threadIdx.x == 0) pd[c + 1] = chi;
                __syncthreads();
                fit_right(XH, PS, RE, t1, hd, pd, c + 1, D);
            }
        }
    }
    // normalise the centre (column 0) and store env k
    double s2 = 0.0;
    for (int t = threadIdx.x; t < 2 * pd[0] * pd[1]; t += blockDim.x) {
        const int r = t / pd[1], b = t % pd[1];
        s2 += PS[r * ld + b] * PS[r * ld + b];
    }
    s2 = tn_block_sum(s2, red);
    const double nrm0 = sqrt(s2);
    const double inv = nrm0 > 0.0 ? 1.0 / nrm0 : 0.0;
    double *Ek = dsc.env + (size_t)k * Lx * 2 * D * D;
    for (size_t t = threadIdx.x; t < (size_t)Lx * 2 * D * D; t += blockDim.x) {
        const int c = (int)(t / (2 * D * D));
        const int rem = (int)(t % (2 * D * D));
        const int a = rem / (2 * D), u = (rem / D) & 1, b = rem % D;
        double v = 0.0;
        if (a < pd[c] && b < pd[c + 1]) v = PS[c * box + (a * 2 + u) * ld + b] * (c == 0 ? inv : 1.0);
        Ek[t] = v;
    }
    for (int c = threadIdx.x; c <= Lx; c += blockDim.x) dsc.dims[k * (Lx + 1) + c] = c < Lx ? pd[c] : 1;
    if (threadIdx.x == 0) {
        dsc.ell[k] = lnqr + log(nrm0);
        dsc.cst[k] = -1;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_env_fit(const tn_env_desc *__restrict__ descs, int step) {
    extern __shared__ double lds[];
    const tn_env_desc dsc = descs[blockIdx.x];
    const int k = dsc.Ly - 1 - step;
    if (k < 1 || dsc.fit <= 0) return;
    fit_row(dsc, k, lds);
}

// Row step `step` of every instance (row k = Ly - 1 - step; the instances
// that have no such row return at once): the MPO application and the
// compression of row k.
// One kernel per class of bond cap (the instances of the other class return
// at once): D <= 32 with 512 threads and the work matrices in LDS, D 33-64
// with 1024 threads (one 16-lane row per row pair of the 2 D-row SVD matrix).
// The kernels for D <= 32 are held to 128 VGPRs (four waves per SIMD), so
// that several workgroups share a compute unit when many instances build
// together; they need no spills for that.  D <= 16 takes 256 threads: its
// Jacobi rounds have at most 16 row pairs, one per 16-lane row, and four of
// its workgroups fit a compute unit's LDS.
// Frozen truncation of row k (the contraction whose derivative tn_grad
// takes): the MPO-MPS product X in xbox is replaced by P X, P the orthogonal
// projector onto span{|columns 0..c*-1> x |columns c*.. of the frozen env k>},
// c* = pcst[k] the leftmost column whose left bond that build truncated.  The
// overlap O of X's columns c*.. with the frozen env's (right-orthonormal)
// columns is carried right to left, rescaled by its largest entry at every
// column, and absorbed into column c*-1; columns c*.. become the frozen env's.
// Returns ln of the removed scale.  Scratch (pscr, 8 D^2 doubles):
// O [2D][D], T [2D][2][D], On [2D][D].
__device__ double project_row(const tn_env_desc &dsc, int k) {
    const int c0 = dsc.pcst[k];
    if (c0 < 1) return 0.0;   // nothing was truncated: the identity
    const int Lx = dsc.Lx, D = dsc.D, ld = 2 * D;
    const size_t box = (size_t)8 * D * D, ebox = (size_t)2 * D * D;
    double *xbox = dsc.xbox;
    int *xdims = dsc.xdims;
    const int *pd = dsc.pdims + (size_t)k * (Lx + 1);
    const double *Ek = dsc.penv + (size_t)k * Lx * ebox;
    double *O = dsc.pscr, *T = O + 2 * D * D, *On = T + 4 * D * D;
    __shared__ double red[16];
    __shared__ int om;   // rows of O (the left bond of X at the current column)
    if (threadIdx.x == 0) {
        O[0] = 1.0;
        om = 1;
    }
    __syncthreads();
    double logscale = 0.0;
    for (int c = Lx - 1; c >= c0; --c) {
        const double *X = xbox + c * box;
        const double *E = Ek + c * ebox;
        const int m = xdims[c], n = xdims[Lx + 1 + c], pl = pd[c], pr = pd[c + 1];
        // T[a][u][d] = sum_b X_c[a][u][b] O[b][d]   (b < n = rows of O)
        for (int t = threadIdx.x; t < m * 2 * pr; t += blockDim.x) {
            const int a = t / (2 * pr), u = (t / pr) & 1, d = t % pr;
            double acc = 0.0;
            for (int b = 0; b < n; ++b) acc += X[(a * 2 + u) * ld + b] * O[b * D + d];
            T[(a * 2 + u) * D + d] = acc;
        }
        __syncthreads();
        // On[a][e] = sum_{u,d} T[a][u][d] E_c[e][u][d]
        double mx = 0.0;
        for (int t = threadIdx.x; t < m * pl; t += blockDim.x) {
            const int a = t / pl, e = t % pl;
            double acc = 0.0;
            for (int u = 0; u < 2; ++u)
                for (int d = 0; d < pr; ++d) acc += T[(a * 2 + u) * D + d] * E[e * 2 * D + u * D + d];
            On[a * D + e] = acc;
            mx = fmax(mx, fabs(acc));
        }
        mx = tn_block_max(mx, red);
        const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
        if (mx > 0.0) logscale += log(mx);
        for (int t = threadIdx.x; t < m * pl; t += blockDim.x) O[(t / pl) * D + t % pl] = On[(t / pl) * D + t % pl] * inv;
        if (threadIdx.x == 0) om = m;
        __syncthreads();
    }
    // X_{c*-1}[a][u][e] = sum_b X_{c*-1}[a][u][b] O[b][e]
    {
        double *X = xbox + (c0 - 1) * box;
        const int m1 = xdims[c0 - 1], n1 = om, pe = pd[c0];
        for (int t = threadIdx.x; t < m1 * 2 * pe; t += blockDim.x) {
            const int r = t / pe, e = t % pe;
            double acc = 0.0;
            for (int b = 0; b < n1; ++b) acc += X[r * ld + b] * O[b * D + e];
            T[r * D + e] = acc;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < m1 * 2 * pe; t += blockDim.x) X[(t / pe) * ld + t % pe] = T[(t / pe) * D + t % pe];
        if (threadIdx.x == 0) xdims[Lx + 1 + c0 - 1] = pe;
    }
    // columns c*.. of the frozen env
    for (int c = c0; c < Lx; ++c) {
        double *X = xbox + c * box;
        const double *E = Ek + c * ebox;
        const int pl = pd[c], pr = pd[c + 1];
        for (int t = threadIdx.x; t < pl * 2 * pr; t += blockDim.x) {
            const int e = t / (2 * pr), u = (t / pr) & 1, d = t % pr;
            X[(e * 2 + u) * ld + d] = E[e * 2 * D + u * D + d];
        }
        if (threadIdx.x == 0) {
            xdims[c] = pl;
            xdims[Lx + 1 + c] = pr;
        }
    }
    __syncthreads();
    return logscale;
}

template <int NTH>
__global__ void __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(NTH == 1024 ? 1 : 4, 8)))
k_env_row(const tn_env_desc *__restrict__ descs, int step) {
    extern __shared__ double lds[];
    const tn_env_desc dsc = descs[blockIdx.x];
    const int k = dsc.Ly - 1 - step;
    if (k < 1 || tn_env_class_threads(dsc.D) != NTH) return;
    if (step == 0)   // trivial env below the last row: bond 1 everywhere
        for (int c = threadIdx.x; c <= dsc.Lx; c += blockDim.x) dsc.dims[(size_t)dsc.Ly * (dsc.Lx + 1) + c] = 1;
    mpo_apply_row(dsc, k);
    const double lp = dsc.penv ? project_row(dsc, k) : 0.0;
    truncate_row<NTH < 1024>(dsc, k, lds, lp);
}

// ln <top|env_1>: row 0 (no up legs) contracted with env 1 left to right,
// rescaled by its largest entry after every column.  out[0] = ln|value|,
// out[1] = sign.
__device__ void top_overlap(const tn_env_desc &dsc) {
    const int Lx = dsc.Lx, Ly = dsc.Ly, D = dsc.D;
    const double beta = dsc.beta;
    const double *Jh = dsc.Jh, *Jv = dsc.Jv, *h = dsc.h, *env = dsc.env;
    const int *dims = dsc.dims;
    double *out = dsc.scal;
    __shared__ double st[2][TN_MAX_D], nst[2][TN_MAX_D];
    __shared__ double M[2][2][2];   // [l][d][x]
    __shared__ double red[4];
    const bool triv = (Ly == 1);
    if (threadIdx.x < 2 * TN_MAX_D) {
        (&st[0][0])[threadIdx.x] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) st[0][0] = 1.0;
    double logscale = 0.0;
    for (int c = 0; c < Lx; ++c) {
        const int lw = c > 0 ? 2 : 1, xw = c < Lx - 1 ? 2 : 1, dw = Ly > 1 ? 2 : 1;
        const int Dl = triv ? 1 : dims[1 * (Lx + 1) + c];
        const int Dr = triv ? 1 : dims[1 * (Lx + 1) + c + 1];
        if (threadIdx.x < 8) {
            const int l = (threadIdx.x >> 2) & 1, d = (threadIdx.x >> 1) & 1, x = threadIdx.x & 1;
            double acc = 0.0;
            if (l < lw && d < dw && x < xw) {
                const double hv = h ? h[c] : 0.0;
                for (int s = 0; s < 2; ++s) {
                    const double f = exp(beta * hv * (s ? -1.0 : 1.0));
                    const double ql = c > 0 ? tn_qleg(beta * Jh[c - 1], l, s) : 1.0;
                    const double pr = c < Lx - 1 ? tn_pleg(beta * Jh[c], s, x) : 1.0;
                    const double pd = Ly > 1 ? tn_pleg(beta * Jv[c], s, d) : 1.0;
                    acc += f * ql * pr * pd;
                }
            }
            M[l][d][x] = acc;
        }
        __syncthreads();
        const double *E = env + ((size_t)1 * Lx + c) * 2 * D * D;
        double mx = 0.0;
        for (int t = threadIdx.x; t < xw * Dr; t += blockDim.x) {
            const int x = t / Dr, b = t % Dr;
            double acc = 0.0;
            for (int l = 0; l < lw; ++l)
                for (int a = 0; a < Dl; ++a)
                    for (int d = 0; d < dw; ++d) {
                        const double e = triv ? 1.0 : E[a * 2 * D + d * D + b];
                        acc += st[l][a] * M[l][d][x] * e;
                    }
            nst[x][b] = acc;
            mx = fmax(mx, fabs(acc));
        }
        mx = tn_block_max(mx, red);
        const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
        __syncthreads();
        for (int t = threadIdx.x; t < 2 * TN_MAX_D; t += blockDim.x) {
            const int x = t / TN_MAX_D, b = t % TN_MAX_D;
            st[x][b] = (x < xw && b < Dr) ? nst[x][b] * inv : 0.0;
        }
        if (mx > 0.0) logscale += log(mx);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = st[0][0];
        out[0] = logscale + log(fabs(v));
        out[1] = v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0);
    }
}

__global__ void __launch_bounds__(256) k_env_top(const tn_env_desc *__restrict__ descs) {
    const tn_env_desc dsc = descs[blockIdx.x];
    if (dsc.Ly == 1) {   // trivial env below the only row
        for (int c = threadIdx.x; c <= dsc.Lx; c += blockDim.x) dsc.dims[(size_t)dsc.Ly * (dsc.Lx + 1) + c] = 1;
        __syncthreads();
    }
    top_overlap(dsc);
}

// Outcome of every instance's build, for callers that rebuild many instances
// each step without a host round trip per instance: 0 usable, 1 Z~ not
// positive or ln Z~ not finite, 2 the Jacobi SVD did not converge.  Clears
// the convergence counter for the next build.
__global__ void __launch_bounds__(256) k_env_status(const tn_env_desc *__restrict__ descs, int n,
                                                    int *__restrict__ status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const tn_env_desc d = descs[i];
    double lz = d.scal[0];
    for (int k = 1; k < d.Ly; ++k) lz += d.ell[k];
    const unsigned long long nc = d.counters[CNT_NOCONV];
    d.counters[CNT_NOCONV] = 0ull;
    status[i] = nc ? 2 : ((!(d.scal[1] > 0.0) || !isfinite(lz)) ? 1 : 0);
}

}  // namespace

int tn_env_build_top_status(const tn_build_plan *plan, int *status, hipStream_t stream) {
    if (plan->n <= 0) return TN_OK;
    hipLaunchKernelGGL(k_env_top, dim3(plan->n), dim3(256), 0, stream, plan->dd);
    hipLaunchKernelGGL(k_env_status, dim3((plan->n + 255) / 256), dim3(256), 0, stream, plan->dd, plan->n,
                       status);
    return hipGetLastError() == hipSuccess ? TN_OK : TN_EHIP;
}

int tn_env_build_prepare(tn_ctx *const *ctxs, int n, hipStream_t stream, std::string *err,
                         tn_build_plan *plan) {
    if (n <= 0) return TN_OK;
    tn_ctx *c0 = ctxs[0];
    auto fail = [&](int code, const std::string &msg) {
        if (err) *err = msg;
        return code;
    };
    std::vector<tn_env_desc> ds(n);
    int maxLy = 1, maxD = 1;
    size_t lds_tiny = 0, lds_small = 0, lds_big = 0, lds_fit = 0;   // doubles
    for (int i = 0; i < n; ++i) {
        tn_ctx *ctx = ctxs[i];
        const int Lx = ctx->Lx, Ly = ctx->Ly, D = ctx->D;
        int rc;
        if ((rc = tn_ensure(ctx, (void **)&ctx->xbox, &ctx->xbox_cap,
                            (size_t)Lx * 8 * D * D * sizeof(double))))
            return fail(rc, ctx->err);
        if (D > 32 && (rc = tn_ensure(ctx, (void **)&ctx->wbuf, &ctx->wbuf_cap,
                                      2 * tn_qr_area(D) * sizeof(double))))
            return fail(rc, ctx->err);
        if (!ctx->xdims &&
            hipMalloc((void **)&ctx->xdims, 2 * (4 * TN_MAX_D + 1) * sizeof(int) +
                                                2 * 1024 * sizeof(int)) != hipSuccess)
            return fail(TN_ENOMEM, "hipMalloc failed");
        if (ctx->fit_sweeps > 0) {
            if (D > 32) return fail(TN_EINVAL, "the variational sweeps support D up to 32");
            if ((rc = tn_ensure(ctx, (void **)&ctx->fbuf, &ctx->fbuf_cap,
                                fit_layout(Lx, D).total * sizeof(double))))
                return fail(rc, ctx->err);
            lds_fit = 2 * tn_svd_area(D) > lds_fit ? 2 * tn_svd_area(D) : lds_fit;
        }
        tn_env_desc &d = ds[i];
        d.Lx = Lx;
        d.Ly = Ly;
        d.D = D;
        d.fit = ctx->fit_sweeps;
        d.fbuf = ctx->fbuf;
        d.beta = ctx->beta;
        d.Jh = ctx->Jh;
        d.Jv = ctx->Jv;
        d.h = ctx->h;
        d.env = ctx->env;
        d.dims = ctx->dims;
        d.ell = ctx->ell;
        d.cst = ctx->cst;
        d.xbox = ctx->xbox;
        d.xdims = ctx->xdims;
        d.wbuf = ctx->wbuf;
        d.penv = nullptr;
        d.pdims = nullptr;
        d.pcst = nullptr;
        d.pscr = nullptr;
        if (const tn_ctx *src = ctx->proj_src) {
            if (src->D != D || src->Lx != Lx || src->Ly != Ly || !src->has_cst)
                return fail(TN_EINVAL, "frozen evaluation: the projector build does not match");
            if ((rc = tn_ensure(ctx, (void **)&ctx->pscr, &ctx->pscr_cap, (size_t)8 * D * D * sizeof(double))))
                return fail(rc, ctx->err);
            d.penv = src->env;
            d.pdims = src->dims;
            d.pcst = src->cst;
            d.pscr = ctx->pscr;
        }
        d.scal = ctx->scal;
        d.counters = ctx->counters;
        maxLy = Ly > maxLy ? Ly : maxLy;
        maxD = D > maxD ? D : maxD;
        size_t &lds_cls = D <= 16 ? lds_tiny : (D <= 32 ? lds_small : lds_big);
        const size_t need = D <= 32 ? 2 * tn_qr_area(D) : tn_svd_area(D);
        lds_cls = need > lds_cls ? need : lds_cls;
    }
    int rc;
    if ((rc = tn_ensure(c0, (void **)&c0->descs, &c0->descs_cap, n * sizeof(tn_env_desc))))
        return fail(rc, c0->err);
    tn_env_desc *dd = (tn_env_desc *)c0->descs;
    if (hipMemcpyAsync(dd, ds.data(), n * sizeof(tn_env_desc), hipMemcpyHostToDevice, stream) !=
        hipSuccess)
        return fail(TN_EHIP, "descriptor copy failed");
    for (int i = 0; i < n; ++i)
        if (hipMemsetAsync(ctxs[i]->counters + CNT_NOCONV, 0, sizeof(unsigned long long), stream) !=
            hipSuccess)
            return fail(TN_EHIP, "counter reset failed");
    plan->n = n;
    plan->maxLy = maxLy;
    plan->lds_tiny = lds_tiny * sizeof(double);
    plan->lds_fit = lds_fit * sizeof(double);
    plan->lds_small = lds_small * sizeof(double);
    plan->lds_big = lds_big * sizeof(double);
    plan->dd = dd;
    plan->ms = 0.0;
    return TN_OK;
}

int tn_env_build_steps(tn_build_plan *plan, int s0, int s1, hipStream_t stream, std::string *err) {
    auto t0 = std::chrono::steady_clock::now();
    // the LDS limits, set here (not when the plan is prepared): another plan
    // may have lowered them since
    if ((plan->lds_tiny && hipFuncSetAttribute((const void *)k_env_row<256>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)plan->lds_tiny) != hipSuccess) ||
        (plan->lds_small && hipFuncSetAttribute((const void *)k_env_row<512>,
                                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                                (int)plan->lds_small) != hipSuccess) ||
        (plan->lds_big && hipFuncSetAttribute((const void *)k_env_row<1024>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize,
                                              (int)plan->lds_big) != hipSuccess) ||
        (plan->lds_fit && hipFuncSetAttribute((const void *)k_env_fit, hipFuncAttributeMaxDynamicSharedMemorySize,
                                              (int)plan->lds_fit) != hipSuccess)) {
        if (err) *err = "LDS size not accepted";
        return TN_EHIP;
    }
    for (int step = s0; step < s1 && step + 1 < plan->maxLy; ++step) {
        if (plan->lds_tiny)
            hipLaunchKernelGGL(k_env_row<256>, dim3(plan->n), dim3(256), plan->lds_tiny, stream,
                               plan->dd, step);
        if (plan->lds_small)
            hipLaunchKernelGGL(k_env_row<512>, dim3(plan->n), dim3(512), plan->lds_small, stream,
                               plan->dd, step);
        if (plan->lds_big)
            hipLaunchKernelGGL(k_env_row<1024>, dim3(plan->n), dim3(1024), plan->lds_big, stream,
                               plan->dd, step);
        if (plan->lds_fit)
            hipLaunchKernelGGL(k_env_fit, dim3(plan->n), dim3(256), plan->lds_fit, stream, plan->dd, step);
        if (hipGetLastError() != hipSuccess) {
            if (err) *err = "row kernel launch failed";
            return TN_EHIP;
        }
    }
    if (hipStreamSynchronize(stream) != hipSuccess) {
        if (err) *err = "environment build failed";
        return TN_EHIP;
    }
    plan->ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return TN_OK;
}

int tn_env_build_finish(tn_ctx *const *ctxs, int n, tn_build_plan *plan, hipStream_t stream,
                        std::string *err) {
    auto fail = [&](int code, const std::string &msg) {
        if (err) *err = msg;
        return code;
    };
    const tn_env_desc *dd = plan->dd;
    auto t0 = std::chrono::steady_clock::now();
    hipLaunchKernelGGL(k_env_top, dim3(n), dim3(256), 0, stream, dd);
    if (hipGetLastError() != hipSuccess) return fail(TN_EHIP, "top kernel launch failed");
    if (hipStreamSynchronize(stream) != hipSuccess) return fail(TN_EHIP, "environment build failed");
    plan->ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    const double ms = plan->ms;
    int first_bad = TN_OK;
    for (int i = 0; i < n; ++i) {
        tn_ctx *ctx = ctxs[i];
        const int Ly = ctx->Ly;
        double top[2];
        std::vector<double> ell(Ly + 1, 0.0);
        unsigned long long noconv = 0;
        if (hipMemcpy(top, ctx->scal, 2 * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(ell.data(), ctx->ell, (Ly + 1) * sizeof(double), hipMemcpyDeviceToHost) !=
                hipSuccess ||
            hipMemcpy(&noconv, ctx->counters + CNT_NOCONV, sizeof(noconv), hipMemcpyDeviceToHost) !=
                hipSuccess)
            return fail(TN_EHIP, "result copy failed");
        double lz = top[0];
        for (int k = 1; k < Ly; ++k) lz += ell[k];
        ctx->logZ = lz;
        ctx->env_build_ms = ms;
        if (first_bad == TN_OK) {
            if (noconv) {
                first_bad = TN_ENOCONV;
                if (err) *err = "Jacobi SVD did not converge in 60 sweeps (instance " + std::to_string(i) + ")";
            } else if (!(top[1] > 0.0) || !std::isfinite(lz)) {
                first_bad = TN_ENONPOS;
                if (err) *err = "approximate partition function is not positive (instance " + std::to_string(i) + ")";
            }
        }
    }
    return first_bad;
}


int tn_env_build_many(tn_ctx *const *ctxs, int n, hipStream_t stream, std::string *err) {
    if (n <= 0) return TN_OK;
    tn_build_plan plan;
    int rc;
    if ((rc = tn_env_build_prepare(ctxs, n, stream, err, &plan))) return rc;
    if ((rc = tn_env_build_steps(&plan, 0, plan.maxLy - 1, stream, err))) return rc;
    return tn_env_build_finish(ctxs, n, &plan, stream, err);
}

int tn_env_build_device(tn_ctx *ctx, double *logZ_out) {
    tn_ctx *one[1] = {ctx};
    std::string e;
    const int rc = tn_env_build_many(one, 1, ctx->stream, &e);
    if (rc != TN_OK) return tn_fail(ctx, rc, e);
    if (logZ_out) *logZ_out = ctx->logZ;
    return TN_OK;
}
