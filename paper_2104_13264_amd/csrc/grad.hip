// Derivative of ln Z~ with the truncations frozen (fp64).
//
// Every compression step of the environment build is replaced by the fixed
// orthogonal projector P_k onto the span it kept at its leftmost truncated
// column c*_k (the identity where env k cut nothing), so that
//     Z~_frozen = <top| P_1 TM_1 P_2 TM_2 ... P_{Ly-1} TM_{Ly-1} |.>
// is multilinear in the site tensors of App. A and equals Z~ at the build
// point.  d ln Z~ / d A_site is the site's environment divided by Z~:
//   * rows k above the exact bottom region: <U_k| TM_k |env_{k+1}> with the
//     upper state U_{k+1} = P_{k+1}(U_k TM_k), whose columns from c* on are
//     the stored env tensors and whose first c* columns are made
//     left-canonical by Householder QR (no loss);
//   * rows kb-1..Ly-1, below which every env is exact: one strip with U on
//     top, contracted column by column with exact transfer vectors.
// Both use the same column machinery: a transfer vector V[y][x_0..x_{h-1}][e]
// (U bond, the horizontal leg of each strip row, bond of the env below) is
// carried left-to-right (L) and right-to-left (R) one column at a time, and
// each site's environment is assembled from L, R and the column's other
// tensors.  The chain rule to K = beta J and beta h uses the closed-form bond
// split; d/dJ = beta d/dK.
#include "common.hpp"
#include "linalg.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

#define TN_MAX_LX_G 256
#define TN_MAX_STRIP 10

namespace {

constexpr int UM = 64;   // cap on the bond of the upper state

struct Strip {
    int Lx, Ly, r0, h, NX;      // strip rows r0..r0+h-1, NX = 2^h
    int D, DE, kE;              // env box, padded env bond of the bottom (1: none), env index
    double beta;
    const double *Jh, *Jv, *hf; // couplings and field
    const double *U;            // U[c][UM][2][UM]
    const int *ud;              // U bonds, [Lx+1]
    const double *env;          // env stack (kE >= 1)
    const int *dims;            // env dims
};

__device__ __forceinline__ int edim(const Strip &S, int c) {
    return S.kE >= 1 ? S.dims[S.kE * (S.Lx + 1) + c] : 1;
}
__device__ __forceinline__ double Eval(const Strip &S, int c, int e, int d, int e2) {
    if (S.kE < 1) return (e == 0 && d == 0 && e2 == 0) ? 1.0 : 0.0;
    return S.env[((size_t)S.kE * S.Lx + c) * 2 * S.D * S.D + e * 2 * S.D + d * S.D + e2];
}
__device__ __forceinline__ double Uval(const Strip &S, int c, int y, int u, int z) {
    return S.U[(size_t)c * UM * 2 * UM + (y * 2 + u) * UM + z];
}

// MPO tensor M[l][u][d][x] of site (r,c) (sum over the spin, App. A
// Eq. tensor-general with the field factor) and its derivatives with respect
// to K of the left, right, up, down bond and to beta h; absent legs are
// index 0 with value 1 (and 0 at index 1).
__device__ void site_tensor(int r, int c, int Lx, int Ly, double beta, const double *Jh,
                            const double *Jv, const double *hf, double *M, double *dM) {
    const double hv = hf ? hf[r * Lx + c] : 0.0;
    const bool hl = c > 0, hr = c < Lx - 1, hu = r > 0, hd = r < Ly - 1;
    const double Kl = hl ? beta * Jh[r * (Lx - 1) + c - 1] : 0.0;
    const double Kr = hr ? beta * Jh[r * (Lx - 1) + c] : 0.0;
    const double Ku = hu ? beta * Jv[(r - 1) * Lx + c] : 0.0;
    const double Kd = hd ? beta * Jv[r * Lx + c] : 0.0;
    for (int t = 0; t < 16; ++t) {
        M[t] = 0.0;
        for (int q = 0; q < 5; ++q) dM[q * 16 + t] = 0.0;
    }
    for (int s = 0; s < 2; ++s) {
        const double sv = s ? -1.0 : 1.0;
        const double f = exp(beta * hv * sv);
        double L[2], R[2], Uu[2], Dd[2], dL[2], dR[2], dU[2], dD[2];
        for (int m = 0; m < 2; ++m) {
            L[m] = hl ? tn_qleg(Kl, m, s) : (m == 0 ? 1.0 : 0.0);
            R[m] = hr ? tn_pleg(Kr, s, m) : (m == 0 ? 1.0 : 0.0);
            Uu[m] = hu ? tn_qleg(Ku, m, s) : (m == 0 ? 1.0 : 0.0);
            Dd[m] = hd ? tn_pleg(Kd, s, m) : (m == 0 ? 1.0 : 0.0);
        }
        // d/dK of P(s,0) = Q(0,s) = sqrt(cosh K): sinh K / (2 sqrt(cosh K));
        // of P(s,1) = s sqrt|sinh K|: sign(K) s cosh K / (2 sqrt|sinh K|);
        // of Q(1,s) = sign(K) s sqrt|sinh K|: s cosh K / (2 sqrt|sinh K|)
        auto d0 = [](double K) { return sinh(K) / (2.0 * sqrt(cosh(K))); };
        auto d1 = [](double K) { return cosh(K) / (2.0 * sqrt(fabs(sinh(K)))); };
        dL[0] = hl ? d0(Kl) : 0.0;
        dL[1] = hl ? sv * d1(Kl) : 0.0;
        dR[0] = hr ? d0(Kr) : 0.0;
        dR[1] = hr ? (Kr >= 0.0 ? 1.0 : -1.0) * sv * d1(Kr) : 0.0;
        dU[0] = hu ? d0(Ku) : 0.0;
        dU[1] = hu ? sv * d1(Ku) : 0.0;
        dD[0] = hd ? d0(Kd) : 0.0;
        dD[1] = hd ? (Kd >= 0.0 ? 1.0 : -1.0) * sv * d1(Kd) : 0.0;
        for (int l = 0; l < 2; ++l)
            for (int u = 0; u < 2; ++u)
                for (int d = 0; d < 2; ++d)
                    for (int x = 0; x < 2; ++x) {
                        const int t = ((l * 2 + u) * 2 + d) * 2 + x;
                        M[t] += f * L[l] * R[x] * Uu[u] * Dd[d];
                        dM[0 * 16 + t] += f * dL[l] * R[x] * Uu[u] * Dd[d];
                        dM[1 * 16 + t] += f * L[l] * dR[x] * Uu[u] * Dd[d];
                        dM[2 * 16 + t] += f * L[l] * R[x] * dU[u] * Dd[d];
                        dM[3 * 16 + t] += f * L[l] * R[x] * Uu[u] * dD[d];
                        dM[4 * 16 + t] += sv * f * L[l] * R[x] * Uu[u] * Dd[d];
                    }
    }
}

// ---- column steps (one workgroup; every thread takes part; ends synced)
// vector V[y][xb][e] flat ((y*NX)+xb)*DE+e; tensors T[v][y][xb][e] = v*VS + ...

__device__ void step_U_left(const Strip &S, int c, const double *V, double *T, int VS) {
    const int dUl = S.ud[c], dUr = S.ud[c + 1], dEl = edim(S, c);
    const int n = 2 * dUr * S.NX * dEl;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int e = t % dEl, xb = (t / dEl) % S.NX, z = (t / (dEl * S.NX)) % dUr,
                  u = t / (dEl * S.NX * dUr);
        double acc = 0.0;
        for (int y = 0; y < dUl; ++y)
            acc += V[((size_t)y * S.NX + xb) * S.DE + e] * Uval(S, c, y, u, z);
        T[(size_t)u * VS + ((size_t)z * S.NX + xb) * S.DE + e] = acc;
    }
    __syncthreads();
}

// apply site j of the column: (x_j, v_j) -> (x'_j, v_{j+1}) (left) or the
// transposed map (right); Mj is [l][u][d][x]
__device__ void step_site(const Strip &S, int c, int j, const double *Mj, const double *Tin,
                          double *Tout, int VS, int dY, int dE, bool left) {
    const int n = 2 * dY * S.NX * dE;
    const int bit = 1 << j;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int e = t % dE, xb = (t / dE) % S.NX, y = (t / (dE * S.NX)) % dY,
                  vo = t / (dE * S.NX * dY);
        const int xo = (xb & bit) ? 1 : 0;
        double acc = 0.0;
        for (int xi = 0; xi < 2; ++xi) {
            const int xbi = (xb & ~bit) | (xi ? bit : 0);
            for (int vi = 0; vi < 2; ++vi) {
                // left: out (d=vo, x'=xo) from in (l=xi, u=vi); right: out (u=vo, l=xo) from in (d=vi, x'=xi)
                const double m = left ? Mj[((xi * 2 + vi) * 2 + vo) * 2 + xo]
                                      : Mj[((xo * 2 + vo) * 2 + vi) * 2 + xi];
                acc += m * Tin[(size_t)vi * VS + ((size_t)y * S.NX + xbi) * S.DE + e];
            }
        }
        Tout[(size_t)vo * VS + ((size_t)y * S.NX + xb) * S.DE + e] = acc;
    }
    __syncthreads();
}

__device__ void step_E_left(const Strip &S, int c, const double *T, double *V) {
    const int dUr = S.ud[c + 1], dEl = edim(S, c), dEr = edim(S, c + 1);
    const int VS = UM * S.NX * S.DE;
    const int n = dUr * S.NX * dEr;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int e2 = t % dEr, xb = (t / dEr) % S.NX, z = t / (dEr * S.NX);
        double acc = 0.0;
        for (int d = 0; d < 2; ++d)
            for (int e = 0; e < dEl; ++e)
                acc += T[(size_t)d * VS + ((size_t)z * S.NX + xb) * S.DE + e] * Eval(S, c, e, d, e2);
        V[((size_t)z * S.NX + xb) * S.DE + e2] = acc;
    }
    __syncthreads();
}

__device__ void step_E_right(const Strip &S, int c, const double *W, double *T) {
    const int dUr = S.ud[c + 1], dEl = edim(S, c), dEr = edim(S, c + 1);
    const int VS = UM * S.NX * S.DE;
    const int n = 2 * dUr * S.NX * dEl;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int e = t % dEl, xb = (t / dEl) % S.NX, z = (t / (dEl * S.NX)) % dUr,
                  d = t / (dEl * S.NX * dUr);
        double acc = 0.0;
        for (int e2 = 0; e2 < dEr; ++e2)
            acc += W[((size_t)z * S.NX + xb) * S.DE + e2] * Eval(S, c, e, d, e2);
        T[(size_t)d * VS + ((size_t)z * S.NX + xb) * S.DE + e] = acc;
    }
    __syncthreads();
}

__device__ void step_U_right(const Strip &S, int c, const double *T, double *W) {
    const int dUl = S.ud[c], dUr = S.ud[c + 1], dEl = edim(S, c);
    const int VS = UM * S.NX * S.DE;
    const int n = dUl * S.NX * dEl;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int e = t % dEl, xb = (t / dEl) % S.NX, y = t / (dEl * S.NX);
        double acc = 0.0;
        for (int u = 0; u < 2; ++u)
            for (int z = 0; z < dUr; ++z)
                acc += T[(size_t)u * VS + ((size_t)z * S.NX + xb) * S.DE + e] * Uval(S, c, y, u, z);
        W[((size_t)y * S.NX + xb) * S.DE + e] = acc;
    }
    __syncthreads();
}

__device__ void rescale(double *V, int dY, int NX, int DE, int dE, double *red) {
    const int n = dY * NX * dE;
    double m = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int e = t % dE, rest = t / dE;
        m = fmax(m, fabs(V[(size_t)rest * DE + e]));
    }
    m = tn_block_max(m, red);
    const double inv = m > 0.0 ? 1.0 / m : 1.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int e = t % dE, rest = t / dE;
        V[(size_t)rest * DE + e] *= inv;
    }
    __syncthreads();
}

// Transfer vectors of the strip: vec[c] for c = 0..Lx (left of column c when
// dir = 0, right of column c-1 when dir = 1).  work: 2 buffers of 2*VS.
__global__ void __launch_bounds__(1024)
k_strip_sweep(Strip S, int dir, double *__restrict__ vec, double *__restrict__ work) {
    __shared__ double M[16], dM[80];
    __shared__ double red[16];
    const int VS = UM * S.NX * S.DE;
    double *A = work, *B = work + 2 * (size_t)VS;
    if (dir == 0) {
        double *V0 = vec;
        for (int t = threadIdx.x; t < VS; t += blockDim.x) V0[t] = (t == 0) ? 1.0 : 0.0;
        __syncthreads();
        for (int c = 0; c < S.Lx; ++c) {
            const double *V = vec + (size_t)c * VS;
            step_U_left(S, c, V, A, VS);
            double *in = A, *out = B;
            for (int j = 0; j < S.h; ++j) {
                if (threadIdx.x == 0) site_tensor(S.r0 + j, c, S.Lx, S.Ly, S.beta, S.Jh, S.Jv, S.hf, M, dM);
                __syncthreads();
                step_site(S, c, j, M, in, out, VS, S.ud[c + 1], edim(S, c), true);
                double *tmp = in;
                in = out;
                out = tmp;
            }
            double *Vn = vec + (size_t)(c + 1) * VS;
            step_E_left(S, c, in, Vn);
            rescale(Vn, S.ud[c + 1], S.NX, S.DE, edim(S, c + 1), red);
        }
    } else {
        double *W0 = vec + (size_t)S.Lx * VS;
        for (int t = threadIdx.x; t < VS; t += blockDim.x) W0[t] = (t == 0) ? 1.0 : 0.0;
        __syncthreads();
        for (int c = S.Lx - 1; c >= 0; --c) {
            const double *W = vec + (size_t)(c + 1) * VS;
            step_E_right(S, c, W, A);
            double *in = A, *out = B;
            for (int j = S.h - 1; j >= 0; --j) {
                if (threadIdx.x == 0) site_tensor(S.r0 + j, c, S.Lx, S.Ly, S.beta, S.Jh, S.Jv, S.hf, M, dM);
                __syncthreads();
                step_site(S, c, j, M, in, out, VS, S.ud[c + 1], edim(S, c), false);
                double *tmp = in;
                in = out;
                out = tmp;
            }
            double *Wn = vec + (size_t)c * VS;
            step_U_right(S, c, in, Wn);
            rescale(Wn, S.ud[c], S.NX, S.DE, edim(S, c), red);
        }
    }
}

// Site environments of column c = blockIdx.x; dsite[r][c][q] receives
// <g, dM_q> / <g, M> for q = left, right, up, down bond and field.
// work per column: (h + 3) buffers of 2*VS.
__global__ void __launch_bounds__(256)
k_strip_sites(Strip S, const double *__restrict__ Lvec, const double *__restrict__ Rvec,
              double *__restrict__ work, double *__restrict__ dsite) {
    const int c = blockIdx.x;
    const int VS = UM * S.NX * S.DE;
    const size_t BUF = 2 * (size_t)VS;
    double *wk = work + (size_t)c * (S.h + 3) * BUF;
    double *Bb = wk;                              // B_1..B_h at Bb + (j-1)*BUF
    double *Ta = wk + (size_t)S.h * BUF, *Tb = Ta + BUF, *Tc = Tb + BUF;
    __shared__ double Ms[TN_MAX_STRIP][16], dMs[TN_MAX_STRIP][80];
    __shared__ double part[4][16];
    __shared__ double red[4];
    if (threadIdx.x < S.h)
        site_tensor(S.r0 + threadIdx.x, c, S.Lx, S.Ly, S.beta, S.Jh, S.Jv, S.hf, Ms[threadIdx.x],
                    dMs[threadIdx.x]);
    __syncthreads();
    const int dUr = S.ud[c + 1], dEl = edim(S, c);
    // B_h = E applied to R; B_j = site j applied (transposed) to B_{j+1}
    step_E_right(S, c, Rvec + (size_t)(c + 1) * VS, Bb + (size_t)(S.h - 1) * BUF);
    for (int j = S.h - 1; j >= 1; --j)
        step_site(S, c, j, Ms[j], Bb + (size_t)j * BUF, Bb + (size_t)(j - 1) * BUF, VS, dUr, dEl,
                  false);
    // T_0 = U applied to L; T_{j+1} = site j applied to T_j
    step_U_left(S, c, Lvec + (size_t)c * VS, Ta, VS);
    double *T = Ta, *Tn = Tb;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int j = 0; j < S.h; ++j) {
        const double *Bj = Bb + (size_t)j * BUF;   // B_{j+1}: sites > j applied
        const int bit = 1 << j;
        double acc[16];
        for (int q = 0; q < 16; ++q) acc[q] = 0.0;
        const int n = dUr * (S.NX / 2) * dEl;
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            const int e = t % dEl, xr = (t / dEl) % (S.NX / 2), z = t / (dEl * (S.NX / 2));
            const int lo = xr & (bit - 1), hi = (xr >> j) << (j + 1);
            const int xb0 = hi | lo, xb1 = xb0 | bit;
            const size_t o0 = ((size_t)z * S.NX + xb0) * S.DE + e, o1 = ((size_t)z * S.NX + xb1) * S.DE + e;
            for (int l = 0; l < 2; ++l)
                for (int u = 0; u < 2; ++u) {
                    const double tv = T[(size_t)u * VS + (l ? o1 : o0)];
                    for (int d = 0; d < 2; ++d)
                        for (int x = 0; x < 2; ++x)
                            acc[((l * 2 + u) * 2 + d) * 2 + x] += tv * Bj[(size_t)d * VS + (x ? o1 : o0)];
                }
        }
        for (int q = 0; q < 16; ++q) {
            const double v = tn_wave_sum(acc[q]);
            if (lane == 0) part[w][q] = v;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double g[16], Z = 0.0;
            for (int q = 0; q < 16; ++q) {
                g[q] = part[0][q] + part[1][q] + part[2][q] + part[3][q];
                Z += g[q] * Ms[j][q];
            }
            double *out = dsite + ((size_t)(S.r0 + j) * S.Lx + c) * 5;
            for (int k = 0; k < 5; ++k) {
                double s = 0.0;
                for (int q = 0; q < 16; ++q) s += g[q] * dMs[j][k * 16 + q];
                out[k] = s / Z;
            }
        }
        __syncthreads();
        if (j + 1 < S.h) {
            step_site(S, c, j, Ms[j], T, Tn, VS, dUr, dEl, true);
            double *tmp = T;
            T = Tn;
            Tn = tmp;
        }
    }
    (void)Tc;
    (void)red;
}

// Y_c = U_c TM_k (bra times row MPO), in the box layout of the environment
// build with bond cap UM: rows (y,l) and d, columns (y',x).
__global__ void __launch_bounds__(256)
k_bra_apply(int k, int Lx, int Ly, double beta, const double *__restrict__ Jh,
            const double *__restrict__ Jv, const double *__restrict__ hf,
            const double *__restrict__ U, const int *__restrict__ ud, double *__restrict__ Y,
            int *__restrict__ ydims) {
    const int c = blockIdx.x;
    __shared__ double M[16], dM[80];
    if (threadIdx.x == 0) site_tensor(k, c, Lx, Ly, beta, Jh, Jv, hf, M, dM);
    __syncthreads();
    const int lw = c > 0 ? 2 : 1, xw = c < Lx - 1 ? 2 : 1;
    const int dUl = ud[c], dUr = ud[c + 1];
    const int m = dUl * lw, n = dUr * xw, ld = 2 * UM;
    double *Yc = Y + (size_t)c * 8 * UM * UM;
    for (int t = threadIdx.x; t < m * 2 * n; t += blockDim.x) {
        const int j = t % n, rest = t / n, d = rest & 1, i = rest >> 1;
        const int y = i / lw, l = i % lw, z = j / xw, x = j % xw;
        double acc = 0.0;
        for (int u = 0; u < 2; ++u)
            acc += U[(size_t)c * UM * 2 * UM + (y * 2 + u) * UM + z] * M[((l * 2 + u) * 2 + d) * 2 + x];
        Yc[(i * 2 + d) * ld + j] = acc;
    }
    if (threadIdx.x == 0) {
        ydims[c] = m;
        ydims[Lx + 1 + c] = n;
    }
}

// P_{c*} applied to Y (columns c* .. replaced by env k tensors, their overlap
// absorbed into column c*-1), then a Householder QR sweep over columns
// 0 .. m-2 (m = c*, or Lx without a projector), then U <- Y.  One workgroup.
__global__ void __launch_bounds__(1024)
k_project_qr(int kenv, int cs, int Lx, int D, const double *__restrict__ env,
             const int *__restrict__ dims, double *__restrict__ Y, int *__restrict__ ydims,
             double *__restrict__ gw, double *__restrict__ U, int *__restrict__ ud,
             int *__restrict__ status) {
    __shared__ int mY[TN_MAX_LX_G + 1], nY[TN_MAX_LX_G + 1];
    __shared__ double tau[2 * UM];
    __shared__ double red[16];
    const int ld = 2 * UM;
    const size_t box = (size_t)8 * UM * UM;
    for (int c = threadIdx.x; c < Lx; c += blockDim.x) {
        mY[c] = ydims[c];
        nY[c] = ydims[Lx + 1 + c];
    }
    __syncthreads();
    double *O = gw, *On = gw + 2 * UM * UM, *T = gw + 4 * UM * UM;   // O [2UM][UM]
    int m = Lx;
    if (cs >= 1) {
        m = cs;
        // O_Lx = [[1]]
        if (threadIdx.x == 0) O[0] = 1.0;
        __syncthreads();
        int dOr = 1;   // right dim of O (= env bond at c+1)
        for (int c = Lx - 1; c >= cs; --c) {
            const double *Yc = Y + c * box;
            const double *E = env + ((size_t)kenv * Lx + c) * 2 * D * D;
            const int a_n = mY[c], b_n = nY[c];
            const int eL = dims[kenv * (Lx + 1) + c];
            // T[a][u][e'] = sum_b Y[a][u][b] O[b][e']
            for (int t = threadIdx.x; t < a_n * 2 * dOr; t += blockDim.x) {
                const int e2 = t % dOr, u = (t / dOr) & 1, a = t / (2 * dOr);
                double acc = 0.0;
                for (int b = 0; b < b_n; ++b) acc += Yc[(a * 2 + u) * ld + b] * O[b * UM + e2];
                T[t] = acc;
            }
            __syncthreads();
            // On[a][e] = sum_{u,e'} T[a][u][e'] E[e][u][e']
            for (int t = threadIdx.x; t < a_n * eL; t += blockDim.x) {
                const int e = t % eL, a = t / eL;
                double acc = 0.0;
                for (int u = 0; u < 2; ++u)
                    for (int e2 = 0; e2 < dOr; ++e2)
                        acc += T[(a * 2 + u) * dOr + e2] * E[e * 2 * D + u * D + e2];
                On[a * UM + e] = acc;
            }
            __syncthreads();
            // keep the carried overlap at unit scale (the scale is free)
            double om = 0.0;
            for (int t = threadIdx.x; t < a_n * eL; t += blockDim.x)
                om = fmax(om, fabs(On[(t / eL) * UM + t % eL]));
            om = tn_block_max(om, red);
            if (om > 0.0)
                for (int t = threadIdx.x; t < a_n * eL; t += blockDim.x) On[(t / eL) * UM + t % eL] /= om;
            __syncthreads();
            double *tmp = O;
            O = On;
            On = tmp;
            dOr = eL;
        }
        // column cs-1 absorbs O; columns cs.. become the env tensors
        {
            double *Yc = Y + (cs - 1) * box;
            const int rows = 2 * mY[cs - 1], b_n = nY[cs - 1];
            for (int t = threadIdx.x; t < rows * dOr; t += blockDim.x) {
                const int e = t % dOr, r = t / dOr;
                double acc = 0.0;
                for (int b = 0; b < b_n; ++b) acc += Yc[r * ld + b] * O[b * UM + e];
                T[t] = acc;
            }
            __syncthreads();
            for (int t = threadIdx.x; t < rows * dOr; t += blockDim.x) {
                const int e = t % dOr, r = t / dOr;
                Yc[r * ld + e] = T[t];
            }
            if (threadIdx.x == 0) nY[cs - 1] = dOr;
        }
        for (int c = cs; c < Lx; ++c) {
            const double *E = env + ((size_t)kenv * Lx + c) * 2 * D * D;
            const int eL = dims[kenv * (Lx + 1) + c], eR = dims[kenv * (Lx + 1) + c + 1];
            double *Yc = Y + c * box;
            for (int t = threadIdx.x; t < eL * 2 * eR; t += blockDim.x) {
                const int e2 = t % eR, u = (t / eR) & 1, e = t / (2 * eR);
                Yc[(e * 2 + u) * ld + e2] = E[e * 2 * D + u * D + e2];
            }
            if (threadIdx.x == 0) {
                mY[c] = eL;
                nY[c] = eR;
            }
        }
        __syncthreads();
    }
    // QR sweep over columns 0 .. m-2: X_c <- Q, X_{c+1} <- R X_{c+1}
    double *W = gw + 6 * UM * UM, *Q = W + 8 * UM * UM;
    for (int c = 0; c + 1 < m; ++c) {
        double *X = Y + c * box, *Xn = Y + (c + 1) * box;
        const int rows = 2 * mY[c], n = nY[c], n1 = nY[c + 1];
        for (int t = threadIdx.x; t < rows * n; t += blockDim.x) W[t] = X[(t / n) * ld + t % n];
        __syncthreads();
        wg_householder(W, rows, n, tau);
        const int kk = min(rows, n);
        wg_form_q(W, rows, n, tau, Q, kk);
        for (int t = threadIdx.x; t < rows * kk; t += blockDim.x) X[(t / kk) * ld + t % kk] = Q[t];
        __syncthreads();
        for (int t = threadIdx.x; t < kk * 2 * n1; t += blockDim.x) {
            const int p = t / (2 * n1), rem = t % (2 * n1), u = rem / n1, j = rem % n1;
            double acc = 0.0;
            for (int q = p; q < n; ++q) acc += W[p * n + q] * Xn[(q * 2 + u) * ld + j];
            Q[t] = acc;
        }
        __syncthreads();
        double xm = 0.0;
        for (int t = threadIdx.x; t < kk * 2 * n1; t += blockDim.x) xm = fmax(xm, fabs(Q[t]));
        xm = tn_block_max(xm, red);
        const double xinv = xm > 0.0 ? 1.0 / xm : 1.0;
        for (int t = threadIdx.x; t < kk * 2 * n1; t += blockDim.x) {
            const int p = t / (2 * n1), rem = t % (2 * n1), u = rem / n1, j = rem % n1;
            Xn[(p * 2 + u) * ld + j] = Q[t] * xinv;
        }
        if (threadIdx.x == 0) {
            mY[c + 1] = kk;
            nY[c] = kk;
        }
        __syncthreads();
    }
    // bonds must fit the upper-state cap
    if (threadIdx.x == 0) {
        int ok = 1;
        for (int c = 0; c < Lx; ++c) ok &= (mY[c] <= UM && nY[c] <= UM);
        status[0] = ok;
    }
    __syncthreads();
    if (!status[0]) return;
    // U <- Y.  After the sweep the columns left of m - 1 are isometries and
    // those from m on are env tensors, so the state's scale sits in column
    // m - 1 alone: divide that column by its largest entry.  The derivative
    // is a ratio of two contractions of the same upper state, so the scale is
    // free; without it the state grows by the row's partition-function ratio
    // every row and leaves the fp64 range.
    const int cn = m - 1;
    double mx = 0.0;
    for (int t = threadIdx.x; t < mY[cn] * 2 * nY[cn]; t += blockDim.x) {
        const int j = t % nY[cn], r = t / nY[cn];
        mx = fmax(mx, fabs(Y[cn * box + r * ld + j]));
    }
    mx = tn_block_max(mx, red);
    const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
    for (size_t t = threadIdx.x; t < (size_t)Lx * 2 * UM * UM; t += blockDim.x) {
        const int c = (int)(t / (2 * UM * UM));
        const int rem = (int)(t % (2 * UM * UM));
        const int y = rem / (2 * UM), u = (rem / UM) & 1, z = rem % UM;
        double v = 0.0;
        if (y < mY[c] && z < nY[c]) v = Y[c * box + (y * 2 + u) * ld + z] * (c == cn ? inv : 1.0);
        U[t] = v;
    }
    for (int c = threadIdx.x; c <= Lx; c += blockDim.x) ud[c] = c < Lx ? mY[c] : 1;
}

// Upper state of row r for the two-sided estimate: env kf of the upside-down
// lattice (its rows 0..r-1, kf = Ly - r), one column per workgroup.  Upside
// down, the vertical bond above row r has its P factor on the row-r site and
// Q on the row r-1 site, so the open leg carries Q(mu, s_{r-1}); row r's own
// tensor carries Q(mu, s_r) on its up leg.  P(s, mu) = sign(K)^mu Q(mu, s), so
// multiplying leg mu = 1 by sign(K) restores the bond weight exp(K s s').
__global__ void k_upper_from_flipped(int Lx, int D, int kf, const double *__restrict__ envf,
                                     const int *__restrict__ dimsf, const double *__restrict__ Jv,
                                     double beta, int r, double *__restrict__ U,
                                     int *__restrict__ ud) {
    const int c = blockIdx.x;
    const int dl = dimsf[kf * (Lx + 1) + c], dr = dimsf[kf * (Lx + 1) + c + 1];
    const double sg = beta * Jv[(size_t)(r - 1) * Lx + c] >= 0.0 ? 1.0 : -1.0;
    const double *E = envf + ((size_t)kf * Lx + c) * 2 * D * D;
    for (int t = threadIdx.x; t < 2 * UM * UM; t += blockDim.x) {
        const int y = t / (2 * UM), u = (t / UM) & 1, z = t % UM;
        double v = 0.0;
        if (y < dl && z < dr) v = E[y * 2 * D + u * D + z] * (u ? sg : 1.0);
        U[(size_t)c * 2 * UM * UM + t] = v;
    }
    if (threadIdx.x == 0) {
        ud[c] = dl;
        if (c == Lx - 1) ud[Lx] = 1;
    }
}

__global__ void k_trivial_upper(int Lx, double *__restrict__ U, int *__restrict__ ud) {
    for (size_t t = blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)Lx * 2 * UM * UM;
         t += gridDim.x * blockDim.x) {
        const int rem = (int)(t % (2 * UM * UM));
        U[t] = rem == 0 ? 1.0 : 0.0;
    }
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c <= Lx; c += gridDim.x * blockDim.x)
        ud[c] = 1;
}

__global__ void k_grad_reduce(int Lx, int Ly, double beta, const double *__restrict__ dsite,
                              double *__restrict__ dJh, double *__restrict__ dJv) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int nh = Ly * (Lx - 1), nv = (Ly - 1) * Lx;
    if (t < nh) {
        const int r = t / (Lx - 1), c = t % (Lx - 1);
        dJh[t] = beta * (dsite[((size_t)r * Lx + c) * 5 + 1] + dsite[((size_t)r * Lx + c + 1) * 5 + 0]);
    } else if (t < nh + nv) {
        const int q = t - nh, r = q / Lx, c = q % Lx;
        dJv[q] = beta * (dsite[((size_t)r * Lx + c) * 5 + 3] + dsite[((size_t)(r + 1) * Lx + c) * 5 + 2]);
    }
}

}  // namespace

int tn_grad_device(tn_ctx *ctx, const tn_ctx *upper, double *dJh, double *dJv, double *dbeta) {
    const bool two = upper != nullptr;
    if (!two && !ctx->has_cst)
        return tn_fail(ctx, TN_ESTATE, "tn_grad needs an environment built by tn_build_env");
    const int Lx = ctx->Lx, Ly = ctx->Ly, D = ctx->D;
    const double beta = ctx->beta;
    // couplings and fields on the host: K = 0 has no derivative of the split
    std::vector<double> hJh((size_t)Ly * (Lx - 1)), hJv((size_t)(Ly - 1) * Lx), hh;
    std::vector<int> cst(Ly + 1);
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (!hJh.empty())
        TN_HIP(ctx, hipMemcpy(hJh.data(), ctx->Jh, hJh.size() * sizeof(double), hipMemcpyDeviceToHost));
    if (!hJv.empty())
        TN_HIP(ctx, hipMemcpy(hJv.data(), ctx->Jv, hJv.size() * sizeof(double), hipMemcpyDeviceToHost));
    if (ctx->h) {
        hh.resize((size_t)Ly * Lx);
        TN_HIP(ctx, hipMemcpy(hh.data(), ctx->h, hh.size() * sizeof(double), hipMemcpyDeviceToHost));
    }
    if (!two)
        TN_HIP(ctx, hipMemcpy(cst.data(), ctx->cst, (Ly + 1) * sizeof(int), hipMemcpyDeviceToHost));
    for (double J : hJh)
        if (beta * J == 0.0) return tn_fail(ctx, TN_EINVAL, "a bond with beta*J = 0 has no derivative");
    for (double J : hJv)
        if (beta * J == 0.0) return tn_fail(ctx, TN_EINVAL, "a bond with beta*J = 0 has no derivative");
    if (Lx > TN_MAX_LX_G) return tn_fail(ctx, TN_EINVAL, "tn_grad supports Lx <= 256");
    // bottom region: rows kb-1 .. Ly-1 with all envs below untruncated (the
    // two-sided estimate takes every row on its own: one-row strips only)
    int kb = Ly;
    for (int k = Ly - 1; k >= 1 && !two; --k) {
        if (cst[k] >= 0) break;
        kb = k;
    }
    const int r0 = kb - 1 < 0 ? 0 : kb - 1;
    const int hb = two ? 1 : Ly - r0;
    if (hb > TN_MAX_STRIP)
        return tn_fail(ctx, TN_EINVAL, "tn_grad: the untruncated bottom region is too tall ("
                                           + std::to_string(hb) + " rows)");
    // scratch layout
    const size_t VS_top = (size_t)UM * 2 * D, VS_bot = (size_t)UM * ((size_t)1 << hb);
    const size_t VS = std::max(VS_top, VS_bot);
    const int hmax = std::max(1, hb);
    const size_t n_vec = 2 * (size_t)(Lx + 1) * VS;                 // L and R vectors
    const size_t n_work = 4 * VS;                                   // sweep ping-pong
    const size_t n_site = (size_t)Lx * (hmax + 3) * 2 * VS;          // per-column buffers
    const size_t n_U = (size_t)Lx * 2 * UM * UM;
    const size_t n_Y = (size_t)Lx * 8 * UM * UM;
    const size_t n_gw = 24 * (size_t)UM * UM;
    const size_t n_ds = (size_t)Ly * Lx * 5;
    const size_t total = n_vec + n_work + n_site + n_U + n_Y + n_gw + n_ds + 2048;
    int rc;
    if ((rc = tn_ensure(ctx, &ctx->gradscr, &ctx->gradscr_cap, total * sizeof(double)))) return rc;
    double *base = (double *)ctx->gradscr;
    double *Lvec = base, *Rvec = Lvec + (Lx + 1) * VS, *work = Rvec + (Lx + 1) * VS;
    double *site = work + n_work, *U = site + n_site, *Y = U + n_U, *gw = Y + n_Y;
    double *dsite = gw + n_gw;
    int *ints = (int *)(dsite + n_ds);
    int *ud = ints, *ydims = ints + 512, *status = ints + 1536;
    hipLaunchKernelGGL(k_trivial_upper, dim3(64), dim3(256), 0, ctx->stream, Lx, U, ud);
    TN_HIP(ctx, hipGetLastError());

    auto run_strip = [&](int r, int h, int kE) -> int {
        Strip S;
        S.Lx = Lx;
        S.Ly = Ly;
        S.r0 = r;
        S.h = h;
        S.NX = 1 << h;
        S.D = D;
        S.DE = kE >= 1 ? D : 1;
        S.kE = kE;
        S.beta = beta;
        S.Jh = ctx->Jh;
        S.Jv = ctx->Jv;
        S.hf = ctx->h;
        S.U = U;
        S.ud = ud;
        S.env = ctx->env;
        S.dims = ctx->dims;
        hipLaunchKernelGGL(k_strip_sweep, dim3(1), dim3(1024), 0, ctx->stream, S, 0, Lvec, work);
        TN_HIP(ctx, hipGetLastError());
        hipLaunchKernelGGL(k_strip_sweep, dim3(1), dim3(1024), 0, ctx->stream, S, 1, Rvec, work);
        TN_HIP(ctx, hipGetLastError());
        hipLaunchKernelGGL(k_strip_sites, dim3(Lx), dim3(256), 0, ctx->stream, S, Lvec, Rvec,
                           site, dsite);
        TN_HIP(ctx, hipGetLastError());
        return TN_OK;
    };

    if (two) {
        // row r between the top-down boundary of rows 0..r-1 (env Ly - r of
        // the upside-down lattice) and env r + 1 of this one
        for (int r = 0; r < Ly; ++r) {
            if (r > 0) {
                hipLaunchKernelGGL(k_upper_from_flipped, dim3(Lx), dim3(256), 0, ctx->stream, Lx, D,
                                   Ly - r, upper->env, upper->dims, ctx->Jv, beta, r, U, ud);
                TN_HIP(ctx, hipGetLastError());
            }
            if ((rc = run_strip(r, 1, r + 1 < Ly ? r + 1 : -1))) return rc;
        }
        kb = 0;   // skips the frozen rows and the bottom strip below
    }
    for (int k = 0; k + 1 < kb; ++k) {
        if ((rc = run_strip(k, 1, k + 1))) return rc;
        hipLaunchKernelGGL(k_bra_apply, dim3(Lx), dim3(256), 0, ctx->stream, k, Lx, Ly, beta,
                           ctx->Jh, ctx->Jv, ctx->h, U, ud, Y, ydims);
        TN_HIP(ctx, hipGetLastError());
        hipLaunchKernelGGL(k_project_qr, dim3(1), dim3(1024), 0, ctx->stream, k + 1, cst[k + 1],
                           Lx, D, ctx->env, ctx->dims, Y, ydims, gw, U, ud, status);
        TN_HIP(ctx, hipGetLastError());
        int ok = 0;
        TN_HIP(ctx, hipMemcpyAsync(&ok, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (!ok)
            return tn_fail(ctx, TN_EINVAL, "tn_grad: upper-state bond above 64 at row " +
                                               std::to_string(k + 1));
    }
    if (!two && (rc = run_strip(r0, hb, -1))) return rc;
    const int nb = Ly * (Lx - 1) + (Ly - 1) * Lx;
    if (nb > 0) {
        hipLaunchKernelGGL(k_grad_reduce, dim3((nb + 255) / 256), dim3(256), 0, ctx->stream, Lx, Ly,
                           beta, dsite, dJh, dJv);
        TN_HIP(ctx, hipGetLastError());
    }
    // d ln Z~ / d beta = sum_b J_b dK_b + sum_i h_i d(beta h_i)
    std::vector<double> ds((size_t)Ly * Lx * 5);
    TN_HIP(ctx, hipMemcpyAsync(ds.data(), dsite, ds.size() * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (dbeta) {
        double db = 0.0;
        for (int r = 0; r < Ly; ++r)
            for (int c = 0; c < Lx; ++c) {
                const double *q = &ds[((size_t)r * Lx + c) * 5];
                if (c + 1 < Lx) db += hJh[r * (Lx - 1) + c] * q[1];
                if (c > 0) db += hJh[r * (Lx - 1) + c - 1] * q[0];
                if (r + 1 < Ly) db += hJv[r * Lx + c] * q[3];
                if (r > 0) db += hJv[(r - 1) * Lx + c] * q[2];
                if (!hh.empty()) db += hh[(size_t)r * Lx + c] * q[4];
            }
        *dbeta = db;
    }
    return TN_OK;
}
