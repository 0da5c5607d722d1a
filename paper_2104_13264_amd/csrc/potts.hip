// q-state Potts models: the method for a general local dimension d.
//
// App. A writes the partition function of any nearest-neighbour model whose
// variables take d values as a contraction of d x d bond matrices
// (Eq. pf_bond_description), splits each by its SVD into two site factors and
// groups them into site tensors (Eq. tensor-general); Sec. 2 notes that the
// sampler carries over to the Potts model.  Here
//     H(s) = - sum_<ij> J_ij delta(s_i, s_j) - sum_i h_i(s_i),  s in 0..d-1,
// W = exp(K delta) with K = beta J, split in closed form through its
// eigenbasis: the uniform vector and Helmert's orthonormal basis of its
// complement,
//     P(s, mu) = e_mu(s) sqrt|lambda_mu|,  Q(mu, s) = sign(lambda_mu) sqrt|lambda_mu| e_mu(s),
//     lambda_0 = e^K - 1 + d,  lambda_mu = e^K - 1 (mu >= 1).
//
// Kernels (one instance, everything fp64):
//   k_potts_tab   the bond factors, site field factors and bond weights
//   k_potts_row   one row of the bottom-up environment build: MPO-MPS
//                 product, Householder QR sweep left to right, one-sided
//                 Jacobi SVD sweep right to left keeping min(D, rows, cols)
//                 singular values ("successive SVD"), env k and ell_k
//   k_potts_top   ln <top|env_1>
//   k_potts_ops   the sampler operands G_c(s) = sum_dn P_down(s, dn) env_{r+1,c}[:, dn, :]
//   k_potts_rows  the sequential draw of one row for every proposal (plain
//                 fp64, snake order), with a d-way categorical conditional:
//                 the smallest value k with u (w_0 + .. + w_{d-1}) < w_0 + .. + w_k
#include "common.hpp"

#include <chrono>
#include <cmath>
#include <vector>

namespace {

// The factorisations split the workgroup into rows of 16 lanes (one per
// column or row pair) with 16-lane reductions.
#define TN_QW ((int)(threadIdx.x >> 4))
#define TN_QL ((int)(threadIdx.x & 15))
#define TN_NQW ((int)(blockDim.x >> 4))

constexpr int TN_POTTS_MAXD = 6;
constexpr int TN_POTTS_MAXBOND = 32;

// Offsets (doubles) of the factor tables.
struct PottsTab {
    size_t F, PH, QH, PV, QV, EKH, EKV, total;
    __host__ __device__ PottsTab(int Lx, int Ly, int d) {
        const size_t dd = (size_t)d * d;
        F = 0;
        PH = F + (size_t)Ly * Lx * d;
        QH = PH + (size_t)Ly * (Lx - 1) * dd;
        PV = QH + (size_t)Ly * (Lx - 1) * dd;
        QV = PV + (size_t)(Ly - 1) * Lx * dd;
        EKH = QV + (size_t)(Ly - 1) * Lx * dd;
        EKV = EKH + (size_t)Ly * (Lx - 1);
        total = EKV + (size_t)(Ly - 1) * Lx + 1;
    }
};

// Work area of the build (doubles): XW = d D is the largest bond of the
// MPO-MPS product, XR = d XW its largest (bond, value) row count.
struct PottsWork {
    int XW, XR;
    size_t box, xbox, A, Qm, S, W, Wo, Z, Y, tau, sv, total;
    __host__ __device__ PottsWork(int Lx, int d, int D) {
        XW = d * D;
        XR = d * XW;
        box = (size_t)XR * XW;
        xbox = 0;
        A = xbox + (size_t)Lx * box;
        Qm = A + box;
        S = Qm + box;
        W = S + box;
        Wo = W + box;
        Z = Wo + box;
        Y = Z + (size_t)XW * D;
        tau = Y + (size_t)XR * D;
        sv = tau + XW;
        total = sv + 2 * (size_t)XW;
    }
};

// Helmert's orthonormal basis of R^d: e_0 uniform, e_m (m >= 1) orthogonal
// to e_0 .. e_{m-1}.
__device__ __forceinline__ double helmert(int s, int mu, int d) {
    if (mu == 0) return 1.0 / sqrt((double)d);
    const double a = 1.0 / sqrt((double)mu * (mu + 1.0));
    return s < mu ? a : (s == mu ? -mu * a : 0.0);
}

__global__ void k_potts_tab(int Lx, int Ly, int d, double beta, const double *__restrict__ Jh,
                            const double *__restrict__ Jv, const double *__restrict__ h,
                            double *__restrict__ tab) {
    const PottsTab T(Lx, Ly, d);
    const int dd = d * d;
    const int nf = Ly * Lx * d, nh = Ly * (Lx - 1), nv = (Ly - 1) * Lx;
    const int total = nf + (nh + nv) * dd + nh + nv;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
        if (t < nf) {
            tab[T.F + t] = h ? exp(beta * h[t]) : 1.0;
            continue;
        }
        int q = t - nf;
        if (q < (nh + nv) * dd) {
            const int bond = q / dd, e = q % dd, s = e / d, mu = e % d;
            const bool hor = bond < nh;
            const double K = beta * (hor ? Jh[bond] : Jv[bond - nh]);
            const double lam = mu == 0 ? expm1(K) + d : expm1(K);
            const double root = sqrt(fabs(lam));
            const double sg = lam > 0.0 ? 1.0 : (lam < 0.0 ? -1.0 : 0.0);
            const double b = helmert(s, mu, d);
            const size_t o = (size_t)(hor ? bond : bond - nh) * dd;
            // P[s][mu] and Q[mu][s] (the same (s, mu) pair, transposed slot)
            tab[(hor ? T.PH : T.PV) + o + s * d + mu] = b * root;
            tab[(hor ? T.QH : T.QV) + o + mu * d + s] = sg * root * b;
            continue;
        }
        q -= (nh + nv) * dd;
        if (q < nh) tab[T.EKH + q] = exp(beta * Jh[q]);
        else tab[T.EKV + (q - nh)] = exp(beta * Jv[q - nh]);
    }
}

struct PottsLegs {
    const double *tab;
    int Lx, Ly, d;
    PottsTab T;
    __device__ PottsLegs(const double *t, int lx, int ly, int dd) : tab(t), Lx(lx), Ly(ly), d(dd), T(lx, ly, dd) {}
    __device__ double F(int r, int c, int s) const { return tab[T.F + ((size_t)r * Lx + c) * d + s]; }
    __device__ double Ql(int r, int c, int l, int s) const {
        return c > 0 ? tab[T.QH + ((size_t)r * (Lx - 1) + c - 1) * d * d + l * d + s] : 1.0;
    }
    __device__ double Pr(int r, int c, int s, int x) const {
        return c < Lx - 1 ? tab[T.PH + ((size_t)r * (Lx - 1) + c) * d * d + s * d + x] : 1.0;
    }
    __device__ double Qu(int r, int c, int u, int s) const {
        return r > 0 ? tab[T.QV + ((size_t)(r - 1) * Lx + c) * d * d + u * d + s] : 1.0;
    }
    __device__ double Pd(int r, int c, int s, int dn) const {
        return r < Ly - 1 ? tab[T.PV + ((size_t)r * Lx + c) * d * d + s * d + dn] : 1.0;
    }
};

// Householder QR of the m x n column-major matrix A (leading dimension lda):
// R in its upper triangle, Q (m x min(m, n), same leading dimension) in Qm.
__device__ void potts_qr(double *A, int m, int n, int lda, double *tau, double *Qm, double *red) {
    const int kk = min(m, n);
    for (int j = 0; j < kk; ++j) {
        double x2 = 0.0;
        for (int i = j + 1 + (int)threadIdx.x; i < m; i += blockDim.x) x2 += A[(size_t)j * lda + i] * A[(size_t)j * lda + i];
        x2 = tn_block_sum(x2, red);   // ends with a barrier
        const double alpha = A[(size_t)j * lda + j];
        double tj = 0.0;
        if (x2 > 0.0) {
            const double beta = -copysign(sqrt(alpha * alpha + x2), alpha);
            tj = (beta - alpha) / beta;
            const double scale = 1.0 / (alpha - beta);
            for (int i = j + 1 + (int)threadIdx.x; i < m; i += blockDim.x) A[(size_t)j * lda + i] *= scale;
            __syncthreads();
            if (threadIdx.x == 0) A[(size_t)j * lda + j] = beta;
        }
        if (threadIdx.x == 0) tau[j] = tj;
        __syncthreads();
        if (tj != 0.0) {
            // columns j+1.. : one 16-lane row per column
            for (int k = j + 1 + TN_QW; k < n; k += TN_NQW) {
                double s = 0.0;
                for (int i = j + 1 + TN_QL; i < m; i += 16) s += A[(size_t)j * lda + i] * A[(size_t)k * lda + i];
                s = tn_row16_sum(s);
                s = tj * (A[(size_t)k * lda + j] + s);
                for (int i = j + 1 + TN_QL; i < m; i += 16) A[(size_t)k * lda + i] -= s * A[(size_t)j * lda + i];
                if (TN_QL == 0) A[(size_t)k * lda + j] -= s;
            }
        }
        __syncthreads();
    }
    // Q = H_0 H_1 .. H_{kk-1} applied to the first kk columns of the identity
    for (int t = threadIdx.x; t < m * kk; t += blockDim.x) {
        const int l = t / m, i = t % m;
        Qm[(size_t)l * lda + i] = i == l ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = kk - 1; j >= 0; --j) {
        const double tj = tau[j];
        if (tj != 0.0) {
            for (int l = j + TN_QW; l < kk; l += TN_NQW) {
                double s = 0.0;
                for (int i = j + 1 + TN_QL; i < m; i += 16) s += A[(size_t)j * lda + i] * Qm[(size_t)l * lda + i];
                s = tn_row16_sum(s);
                s = tj * (Qm[(size_t)l * lda + j] + s);
                for (int i = j + 1 + TN_QL; i < m; i += 16) Qm[(size_t)l * lda + i] -= s * A[(size_t)j * lda + i];
                if (TN_QL == 0) Qm[(size_t)l * lda + j] -= s;
            }
        }
        __syncthreads();
    }
}

// One-sided Jacobi (Hestenes) on the rows of W (rows x len, row-major,
// leading dimension ldw): rotates pairs of rows until all are mutually
// orthogonal; pairs in round-robin order, one 16-lane row per pair.  Rows
// with squared norm <= zero2 are left alone.  Returns the sweeps taken, -1
// without convergence in 60.
__device__ int potts_jacobi(double *W, int rows, int len, int ldw, double zero2, int *flag) {
    const int n2 = rows + (rows & 1);
    const double eps = 2.220446049250313e-16;
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (threadIdx.x == 0) *flag = 0;
        __syncthreads();
        for (int t = 0; t + 1 < n2; ++t) {
            for (int k = TN_QW; k < n2 / 2; k += TN_NQW) {
                const int p = k == 0 ? n2 - 1 : (t + k) % (n2 - 1);
                const int q = (t - k + n2 - 1) % (n2 - 1);
                if (p >= rows || q >= rows) continue;   // the odd player's bye (uniform per 16 lanes)
                double a = 0.0, b = 0.0, g = 0.0;
                for (int e = TN_QL; e < len; e += 16) {
                    const double wp = W[(size_t)p * ldw + e], wq = W[(size_t)q * ldw + e];
                    a += wp * wp;
                    b += wq * wq;
                    g += wp * wq;
                }
                a = tn_row16_sum(a);
                b = tn_row16_sum(b);
                g = tn_row16_sum(g);
                if (a > zero2 && b > zero2 && fabs(g) > 4.0 * eps * sqrt(a * b)) {
                    const double zeta = (b - a) / (2.0 * g);
                    const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
                    for (int e = TN_QL; e < len; e += 16) {
                        const double wp = W[(size_t)p * ldw + e], wq = W[(size_t)q * ldw + e];
                        W[(size_t)p * ldw + e] = cs * wp - sn * wq;
                        W[(size_t)q * ldw + e] = sn * wp + cs * wq;
                    }
                    if (TN_QL == 0) *flag = 1;
                }
            }
            __syncthreads();
        }
        if (*flag == 0) return sweep + 1;
        __syncthreads();
    }
    return -1;
}

// One row k of the bottom-up build (one workgroup): env k from env k+1.
__global__ void __launch_bounds__(256)
k_potts_row(int k, int Lx, int Ly, int d, int D, const double *__restrict__ tab, double *env, int *dims,
            double *ell, double *work, unsigned long long *counters) {
    const PottsLegs G(tab, Lx, Ly, d);
    const PottsWork P(Lx, d, D);
    const int XW = P.XW, XR = P.XR;
    double *xbox = work + P.xbox;
    double *A = work + P.A, *Qm = work + P.Qm, *S = work + P.S, *W = work + P.W, *Wo = work + P.Wo;
    double *Z = work + P.Z, *Y = work + P.Y, *tau = work + P.tau, *sv = work + P.sv;
    __shared__ double M[TN_POTTS_MAXD * TN_POTTS_MAXD * TN_POTTS_MAXD * TN_POTTS_MAXD];
    __shared__ int mX[257], nX[257];
    __shared__ int idx[TN_POTTS_MAXD * TN_POTTS_MAXBOND];
    __shared__ double red[16];
    __shared__ int flag;
    const size_t ebox = (size_t)d * D * D;
    const bool triv = k == Ly - 1;   // below the last row: the trivial env

    // ---- MPO-MPS product X_c[(a, l), u, (b, x)] = sum_dn E[a][dn][b] M[l][u][dn][x]
    for (int c = 0; c < Lx; ++c) {
        const int lw = c > 0 ? d : 1, xw = c < Lx - 1 ? d : 1, dw = triv ? 1 : d;
        const int Dl = triv ? 1 : dims[(k + 1) * (Lx + 1) + c];
        const int Dr = triv ? 1 : dims[(k + 1) * (Lx + 1) + c + 1];
        for (int t = threadIdx.x; t < lw * d * dw * xw; t += blockDim.x) {
            const int x = t % xw, dn = (t / xw) % dw, u = (t / (xw * dw)) % d, l = t / (xw * dw * d);
            double acc = 0.0;
            for (int s = 0; s < d; ++s)
                acc += G.F(k, c, s) * G.Ql(k, c, l, s) * G.Pr(k, c, s, x) * G.Qu(k, c, u, s) * G.Pd(k, c, s, dn);
            M[((l * d + u) * dw + dn) * xw + x] = acc;
        }
        __syncthreads();
        const int m = Dl * lw, n = Dr * xw;
        double *X = xbox + (size_t)c * P.box;
        const double *E = env + ((size_t)(k + 1) * Lx + c) * ebox;
        for (int t = threadIdx.x; t < m * d * n; t += blockDim.x) {
            const int j = t % n, rest = t / n, u = rest % d, i = rest / d;
            const int a = i / lw, l = i % lw, b = j / xw, x = j % xw;
            double acc = 0.0;
            for (int dn = 0; dn < dw; ++dn) {
                const double e = triv ? 1.0 : E[((size_t)a * d + dn) * D + b];
                acc += e * M[((l * d + u) * dw + dn) * xw + x];
            }
            X[(size_t)(i * d + u) * XW + j] = acc;
        }
        if (threadIdx.x == 0) {
            mX[c] = m;
            nX[c] = n;
        }
        __syncthreads();
    }

    // ---- left-to-right QR sweep: X_c <- Q, X_{c+1} <- R X_{c+1} / |X_c|
    double lognorm = 0.0;
    for (int c = 0; c + 1 < Lx; ++c) {
        double *X = xbox + (size_t)c * P.box, *Xn = xbox + (size_t)(c + 1) * P.box;
        const int m = d * mX[c], n = nX[c], n1 = nX[c + 1];
        double x2 = 0.0;
        for (int t = threadIdx.x; t < m * n; t += blockDim.x) {
            const int r = t / n, j = t % n;
            const double v = X[(size_t)r * XW + j];
            A[(size_t)j * XR + r] = v;
            x2 += v * v;
        }
        x2 = tn_block_sum(x2, red);
        const double xn = sqrt(x2);
        const double xinv = xn > 0.0 ? 1.0 / xn : 1.0;
        if (xn > 0.0) lognorm += log(xn);
        potts_qr(A, m, n, XR, tau, Qm, red);
        const int kk = min(m, n);
        for (int t = threadIdx.x; t < m * kk; t += blockDim.x) {
            const int r = t / kk, l = t % kk;
            X[(size_t)r * XW + l] = Qm[(size_t)l * XR + r];
        }
        // stage X_{c+1} as [q][(u, e)] (n rows), then R X_{c+1} into its first kk rows
        const int w1 = d * n1;
        for (int t = threadIdx.x; t < n * w1; t += blockDim.x) {
            const int q = t / w1, e = t % w1;
            S[t] = Xn[(size_t)(q * d + e / n1) * XW + e % n1];
        }
        __syncthreads();
        for (int t = threadIdx.x; t < kk * w1; t += blockDim.x) {
            const int p = t / w1, e = t % w1;
            double acc = 0.0;
            for (int q = p; q < n; ++q) acc += A[(size_t)q * XR + p] * S[(size_t)q * w1 + e];
            Xn[(size_t)(p * d + e / n1) * XW + e % n1] = acc * xinv;
        }
        if (threadIdx.x == 0) {
            mX[c + 1] = kk;
            nX[c] = kk;
        }
        __syncthreads();
    }
    {   // normalise the last column
        double *X = xbox + (size_t)(Lx - 1) * P.box;
        const int m = mX[Lx - 1], n = nX[Lx - 1];
        double s2 = 0.0;
        for (int t = threadIdx.x; t < m * d * n; t += blockDim.x) s2 += X[(size_t)(t / n) * XW + t % n] * X[(size_t)(t / n) * XW + t % n];
        s2 = tn_block_sum(s2, red);
        const double nrm = sqrt(s2), inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
        for (int t = threadIdx.x; t < m * d * n; t += blockDim.x) X[(size_t)(t / n) * XW + t % n] *= inv;
        lognorm += log(nrm);
        __syncthreads();
    }

    // ---- right-to-left SVD sweep, keeping chi = min(D, rows, cols)
    const double eps = 2.220446049250313e-16;
    for (int c = Lx - 1; c >= 1; --c) {
        double *X = xbox + (size_t)c * P.box, *Xp = xbox + (size_t)(c - 1) * P.box;
        const int rows = mX[c], ncol = nX[c], len = d * ncol;
        double f2 = 0.0;
        for (int t = threadIdx.x; t < rows * len; t += blockDim.x) {
            const int i = t / len, e = t % len;
            const double v = X[(size_t)(i * d + e / ncol) * XW + e % ncol];
            W[(size_t)i * XR + e] = v;
            Wo[(size_t)i * XR + e] = v;
            f2 += v * v;
        }
        f2 = tn_block_sum(f2, red);
        const double zero2 = f2 * (len * eps) * (len * eps);
        const int sweeps = potts_jacobi(W, rows, len, XR, zero2, &flag);
        if (sweeps < 0 && threadIdx.x == 0) atomicAdd(&counters[CNT_NOCONV], 1ull);
        for (int i = TN_QW; i < rows; i += TN_NQW) {
            double s2 = 0.0;
            for (int e = TN_QL; e < len; e += 16) s2 += W[(size_t)i * XR + e] * W[(size_t)i * XR + e];
            s2 = tn_row16_sum(s2);
            if (TN_QL == 0) sv[i] = s2 > zero2 ? sqrt(s2) : 0.0;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < rows; i += blockDim.x) {   // descending, ties by row index
            int r = 0;
            const double si = sv[i];
            for (int j = 0; j < rows; ++j) r += (sv[j] > si) || (sv[j] == si && j < i);
            idx[r] = i;
        }
        __syncthreads();
        const int nsv = min(rows, len), chi = min(D, nsv);
        if (threadIdx.x == 0 && chi < nsv && sv[idx[chi - 1]] - sv[idx[chi]] < 1e-12 * sv[idx[0]])
            atomicAdd(&counters[CNT_DEGEN], 1ull);
        // Z = U S = Wo V = Wo W'^T / s, the kept columns
        for (int t = threadIdx.x; t < rows * chi; t += blockDim.x) {
            const int kq = t / rows, r = t % rows, ik = idx[kq];
            const double s = sv[ik];
            double acc = 0.0;
            if (s > 0.0) {
                for (int e = 0; e < len; ++e) acc += Wo[(size_t)r * XR + e] * W[(size_t)ik * XR + e];
                acc /= s;
            }
            Z[(size_t)r * D + kq] = acc;
        }
        __syncthreads();
        // Y = X_{c-1} Z; X_c <- V^T of the kept values
        const int m1 = d * mX[c - 1];
        for (int t = threadIdx.x; t < m1 * chi; t += blockDim.x) {
            const int r = t / chi, kq = t % chi;
            double acc = 0.0;
            for (int q = 0; q < rows; ++q) acc += Xp[(size_t)r * XW + q] * Z[(size_t)q * D + kq];
            Y[t] = acc;
        }
        for (int t = threadIdx.x; t < chi * len; t += blockDim.x) {
            const int kq = t / len, e = t % len, ik = idx[kq];
            const double s = sv[ik];
            X[(size_t)(kq * d + e / ncol) * XW + e % ncol] = s > 0.0 ? W[(size_t)ik * XR + e] / s : 0.0;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < m1 * chi; t += blockDim.x) Xp[(size_t)(t / chi) * XW + t % chi] = Y[t];
        if (threadIdx.x == 0) {
            mX[c] = chi;
            nX[c - 1] = chi;
        }
        __syncthreads();
    }
    {   // normalise column 0
        double *X = xbox;
        const int m = mX[0], n = nX[0];
        double s2 = 0.0;
        for (int t = threadIdx.x; t < m * d * n; t += blockDim.x) s2 += X[(size_t)(t / n) * XW + t % n] * X[(size_t)(t / n) * XW + t % n];
        s2 = tn_block_sum(s2, red);
        const double nrm = sqrt(s2), inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
        for (int t = threadIdx.x; t < m * d * n; t += blockDim.x) X[(size_t)(t / n) * XW + t % n] *= inv;
        lognorm += log(nrm);
        __syncthreads();
    }
    // ---- store env k: boxes [a][u][b] of D x d x D, zero padded
    for (size_t t = threadIdx.x; t < (size_t)Lx * ebox; t += blockDim.x) {
        const int c = (int)(t / ebox);
        const int rem = (int)(t % ebox);
        const int a = rem / (d * D), u = (rem / D) % d, b = rem % D;
        double v = 0.0;
        if (a < mX[c] && b < nX[c]) v = xbox[(size_t)c * P.box + (size_t)(a * d + u) * XW + b];
        env[(size_t)k * Lx * ebox + t] = v;
    }
    for (int c = threadIdx.x; c <= Lx; c += blockDim.x) dims[k * (Lx + 1) + c] = c < Lx ? mX[c] : 1;
    if (threadIdx.x == 0) ell[k] = lognorm;
}

// ln <top|env_1>: row 0 (no up legs) against env 1, left to right, rescaled
// by the largest entry at every column.  out[0] = ln|value|, out[1] = sign.
__global__ void __launch_bounds__(256)
k_potts_top(int Lx, int Ly, int d, int D, const double *__restrict__ tab, const double *__restrict__ env,
            const int *__restrict__ dims, double *out) {
    const PottsLegs G(tab, Lx, Ly, d);
    __shared__ double st[TN_POTTS_MAXD * TN_POTTS_MAXBOND], nst[TN_POTTS_MAXD * TN_POTTS_MAXBOND];
    __shared__ double M[TN_POTTS_MAXD * TN_POTTS_MAXD * TN_POTTS_MAXD];   // [l][dn][x]
    __shared__ double red[16];
    const bool triv = Ly == 1;
    const size_t ebox = (size_t)d * D * D;
    for (int t = threadIdx.x; t < TN_POTTS_MAXD * TN_POTTS_MAXBOND; t += blockDim.x) st[t] = t == 0 ? 1.0 : 0.0;
    __syncthreads();
    double logscale = 0.0;
    for (int c = 0; c < Lx; ++c) {
        const int lw = c > 0 ? d : 1, xw = c < Lx - 1 ? d : 1, dw = triv ? 1 : d;
        const int Dl = triv ? 1 : dims[1 * (Lx + 1) + c], Dr = triv ? 1 : dims[1 * (Lx + 1) + c + 1];
        for (int t = threadIdx.x; t < lw * dw * xw; t += blockDim.x) {
            const int x = t % xw, dn = (t / xw) % dw, l = t / (xw * dw);
            double acc = 0.0;
            for (int s = 0; s < d; ++s) acc += G.F(0, c, s) * G.Ql(0, c, l, s) * G.Pr(0, c, s, x) * G.Pd(0, c, s, dn);
            M[(l * dw + dn) * xw + x] = acc;
        }
        __syncthreads();
        const double *E = env + ((size_t)1 * Lx + c) * ebox;
        double mx = 0.0;
        for (int t = threadIdx.x; t < xw * Dr; t += blockDim.x) {
            const int x = t / Dr, b = t % Dr;
            double acc = 0.0;
            for (int l = 0; l < lw; ++l)
                for (int a = 0; a < Dl; ++a)
                    for (int dn = 0; dn < dw; ++dn) {
                        const double e = triv ? 1.0 : E[((size_t)a * d + dn) * D + b];
                        acc += st[l * TN_POTTS_MAXBOND + a] * M[(l * dw + dn) * xw + x] * e;
                    }
            nst[x * TN_POTTS_MAXBOND + b] = acc;
            mx = fmax(mx, fabs(acc));
        }
        mx = tn_block_max(mx, red);
        const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
        __syncthreads();
        for (int t = threadIdx.x; t < TN_POTTS_MAXD * TN_POTTS_MAXBOND; t += blockDim.x) {
            const int x = t / TN_POTTS_MAXBOND, b = t % TN_POTTS_MAXBOND;
            st[t] = (x < xw && b < Dr) ? nst[t] * inv : 0.0;
        }
        if (mx > 0.0) logscale += log(mx);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = st[0];
        out[0] = logscale + log(fabs(v));
        out[1] = v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0);
    }
}

// G_c(s)[a][b] = sum_dn P_down(s, dn) env_{r+1,c}[a][dn][b] for every row r
// (the trivial env below the last row: G = 1), in both layouts:
// Gr [r][c][s][a][b] and Gc [r][c][s][b][a].
__global__ void k_potts_ops(int Lx, int Ly, int d, int D, const double *__restrict__ tab,
                            const double *__restrict__ env, const int *__restrict__ dims,
                            double *__restrict__ Gr, double *__restrict__ Gc) {
    const PottsLegs G(tab, Lx, Ly, d);
    const size_t DD = (size_t)D * D, ebox = (size_t)d * DD;
    const size_t total = (size_t)Ly * Lx * d * DD;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const int b = (int)(t % D), a = (int)((t / D) % D), s = (int)((t / DD) % d);
        const size_t rc = t / (d * DD);
        const int c = (int)(rc % Lx), r = (int)(rc / Lx);
        double v = 0.0;
        if (r == Ly - 1) {
            v = (a == 0 && b == 0) ? 1.0 : 0.0;
        } else {
            const int Dl = dims[(r + 1) * (Lx + 1) + c], Dr = dims[(r + 1) * (Lx + 1) + c + 1];
            if (a < Dl && b < Dr) {
                const double *E = env + ((size_t)(r + 1) * Lx + c) * ebox;
                for (int dn = 0; dn < d; ++dn) v += G.Pd(r, c, s, dn) * E[((size_t)a * d + dn) * D + b];
            }
        }
        Gr[t] = v;
        Gc[rc * d * DD + (size_t)s * DD + (size_t)b * D + a] = v;
    }
}

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

// Row r of every proposal (a team of T lanes per proposal, lane j holding
// component j of the bond vectors).  Rightward row (the leftward one is its
// mirror image with G^T and the bond to the right):
//   environment sweep c = Lx-1 .. 0:  y_s = G_c(s) r_s, stored;
//       r_s'^(c-1) = sum_s W(s', s) v_c(s) y_s,  W = exp(K delta) of bond (c-1, c),
//       v_c(s) = exp(beta h_c(s)) exp(K_up delta(s_up, s))
//   drawing sweep c = 0 .. Lx-1:  w(s) = v_c(s) W(s_{c-1}, s) <Lam, y_s>; clamp;
//       the cumulative draw; ln q += ln(w_s / sum); Lam <- Lam G_c(s)
template <int T, int PD>
__global__ void __launch_bounds__(256)
k_potts_rows(int r, int B, int Lx, int Ly, int D, const double *__restrict__ Jh, const double *__restrict__ Jv,
             const double *__restrict__ h, const double *__restrict__ tab, const int *__restrict__ dims,
             const double *__restrict__ Grow, const double *__restrict__ Gcol, int8_t *__restrict__ S, int eval,
             double *__restrict__ logq, double *__restrict__ energy, double *__restrict__ gscr, uint32_t k0,
             uint32_t k1, uint64_t first_id, uint64_t step0, const uint64_t *__restrict__ step_base, int per_step,
             uint32_t inst, unsigned long long *__restrict__ counters) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = tid / T, j = tid % T;
    if (b >= B) return;   // whole teams leave together (T divides 64)
    const PottsTab TB(Lx, Ly, PD);
    const int *dm = dims + (size_t)(r + 1) * (Lx + 1);
    const size_t DD = (size_t)D * D;
    const double *Gr = Grow + (size_t)r * Lx * PD * DD;
    const double *Gc = Gcol + (size_t)r * Lx * PD * DD;
    const double *F = tab + TB.F + (size_t)r * Lx * PD;
    const double *ekh = tab + TB.EKH + (size_t)r * (Lx - 1);
    const double *ekv = r > 0 ? tab + TB.EKV + (size_t)(r - 1) * Lx : nullptr;
    double *gs = gscr + (size_t)b * Lx * PD * D;
    const int8_t *up = r > 0 ? S + ((size_t)b * Ly + r - 1) * Lx : nullptr;
    int8_t *row = S + ((size_t)b * Ly + r) * Lx;
    const bool rightward = (r & 1) == 0;

    // field and bond to the fixed value u above (u < 0: no row above), per value
    auto vweight = [&](int c, int s, int u) {
        double v = F[(size_t)c * PD + s];
        if (u == s) v *= ekv[c];
        return v;
    };
    // Full teams with few operands per lane (PD T <= 48) pipeline their
    // loads: the sweep reads a column's operands one column ahead, the draw
    // every value's operands of its column before it draws.  A column's own
    // loads come first, since loads complete in the order they are issued.
    // (two columns of operands in registers at PD T = 48 leave two waves
    // per SIMD, all that a launch of 8192 proposals fills; PD T = 64 would
    // leave one)
    constexpr bool PIPE = PD * T <= 48;
    constexpr int PP = PIPE ? PD : 1, TP = PIPE ? T : 1;
    const bool pipe = PIPE && D == T;
    auto opload = [&](double (&g)[PP][TP], const double *G0) {
#pragma unroll
        for (int s = 0; s < PP; ++s)
#pragma unroll
            for (int k = 0; k < TP; ++k) g[s][k] = G0[s * DD + k * D + j];
    };

    // ---- environment sweep of the free columns, from the far end of the row
    double rv[PD];
#pragma unroll
    for (int s = 0; s < PD; ++s) rv[s] = (j == 0) ? 1.0 : 0.0;
    const double *Gsw = rightward ? Gc : Gr;   // the sweep's layout
    double gv[PP][TP];                         // operands of the column (pipelined)
    if (pipe) opload(gv, Gsw + (size_t)(rightward ? Lx - 1 : 0) * PD * DD);
    for (int t = 0; t < Lx; ++t) {
        const int c = rightward ? Lx - 1 - t : t;
        const int Dl = dm[c], Dr = dm[c + 1];
        const int u = up ? up[c] : -1;
        double y[PD];
#pragma unroll
        for (int s = 0; s < PD; ++s) y[s] = 0.0;
        if (pipe) {
            // the next column's operands (the last column's again at the end)
            const int cn = t + 1 < Lx ? (rightward ? c - 1 : c + 1) : c;
            double gn[PP][TP];
            opload(gn, Gsw + (size_t)cn * PD * DD);
#pragma unroll
            for (int k = 0; k < TP; ++k)
#pragma unroll
                for (int s = 0; s < PP; ++s) y[s] += gv[s][k] * __shfl(rv[s], k, T);
#pragma unroll
            for (int s = 0; s < PP; ++s)
#pragma unroll
                for (int k = 0; k < TP; ++k) gv[s][k] = gn[s][k];
        } else if (D == T) {
            // full teams: G is zero outside Dl x Dr and so are the vector
            // components past the bond, so a fixed T-term product adds exact
            // zeros after the same terms in the same order; unrolled, its
            // shuffles and loads issue together instead of one chain per term
            const double *G0 = (rightward ? Gc : Gr) + (size_t)c * PD * DD;
#pragma unroll
            for (int k = 0; k < T; ++k)
#pragma unroll
                for (int s = 0; s < PD; ++s) y[s] += G0[s * DD + k * D + j] * __shfl(rv[s], k, T);
        } else if (rightward) {   // y_s = G_c(s) r_s
            const double *G0 = Gc + (size_t)c * PD * DD;
            for (int k = 0; k < Dr; ++k) {
#pragma unroll
                for (int s = 0; s < PD; ++s) {
                    const double x = __shfl(rv[s], k, T);
                    if (j < Dl) y[s] += G0[s * DD + k * D + j] * x;
                }
            }
        } else {           // y_s = G_c(s)^T l_s
            const double *G0 = Gr + (size_t)c * PD * DD;
            for (int k = 0; k < Dl; ++k) {
#pragma unroll
                for (int s = 0; s < PD; ++s) {
                    const double x = __shfl(rv[s], k, T);
                    if (j < Dr) y[s] += G0[s * DD + k * D + j] * x;
                }
            }
        }
        if (j < D) {
#pragma unroll
            for (int s = 0; s < PD; ++s) gs[((size_t)c * PD + s) * D + j] = y[s];
        }
        if (t + 1 < Lx) {
            // the bond towards the next column of the sweep
            const double eK = ekh[rightward ? c - 1 : c];
            double sum = 0.0, vy[PD];
#pragma unroll
            for (int s = 0; s < PD; ++s) {
                vy[s] = vweight(c, s, u) * y[s];
                sum += vy[s];
            }
            double mx = 0.0;
#pragma unroll
            for (int s = 0; s < PD; ++s) {
                rv[s] = sum + (eK - 1.0) * vy[s];
                mx = fmax(mx, fabs(rv[s]));
            }
            const int e = pow2_exponent(team_max<T>(mx));
#pragma unroll
            for (int s = 0; s < PD; ++s) rv[s] = ldexp(rv[s], -e);
        }
    }

    // ---- sampling sweep in the row's direction
    double lam = (j == 0) ? 1.0 : 0.0;
    int sprev = 0;
    double lq = 0.0, E = 0.0;
    uint4 blk = make_uint4(0, 0, 0, 0);
    int blk_id = -1;
    for (int t = 0; t < Lx; ++t) {
        const int c = rightward ? t : Lx - 1 - t;
        const int Dl = dm[c], Dr = dm[c + 1];
        const double eKp = t > 0 ? ekh[rightward ? c - 1 : c] : 1.0;   // bond to the previous draw
        const int u = up ? up[c] : -1;
        // the column's stored right environments, its energy terms and, when
        // pipelined, every value's operands of the left product, in that order
        double gy[PD];
#pragma unroll
        for (int s = 0; s < PD; ++s) gy[s] = j < D ? gs[((size_t)c * PD + s) * D + j] : 0.0;
        double hv[PD];
        if (h) {
#pragma unroll
            for (int q = 0; q < PD; ++q) hv[q] = h[((size_t)r * Lx + c) * PD + q];
        }
        const double jh = t > 0 ? Jh[(size_t)r * (Lx - 1) + (rightward ? c - 1 : c)] : 0.0;
        const double jv = up ? Jv[(size_t)(r - 1) * Lx + c] : 0.0;
        double gd[PP][TP];
        if (pipe) opload(gd, (rightward ? Gr : Gc) + (size_t)c * PD * DD);
        double w[PD], cum[PD];
        int nclamp = 0;
#pragma unroll
        for (int s = 0; s < PD; ++s) {
            const double g = gy[s];
            double v = vweight(c, s, u);
            if (t > 0 && sprev == s) v *= eKp;
            w[s] = v * team_sum<T>(lam * g);
            if (w[s] < 0.0) {
                w[s] = 0.0;
                ++nclamp;
            }
        }
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < PD; ++s) {
            acc += w[s];
            cum[s] = acc;
        }
        const bool bad = !(cum[PD - 1] > 0.0 && cum[PD - 1] <= 1.79e308);
        if (bad) {   // no usable weight: the uniform law
#pragma unroll
            for (int s = 0; s < PD; ++s) {
                w[s] = 1.0;
                cum[s] = s + 1.0;
            }
        }
        const double tot = cum[PD - 1];
        if (j == 0) {
            if (nclamp) atomicAdd(&counters[CNT_CLAMPS], (unsigned long long)nclamp);
            if (bad) atomicAdd(&counters[CNT_BOTH], 1ull);
        }
        int s;
        if (eval) {
            s = row[c];
        } else {
            const int i = r * Lx + c;
            if ((i >> 2) != blk_id) {
                blk_id = i >> 2;
                const uint64_t id = first_id + (uint64_t)b % (uint64_t)per_step;
                const uint32_t st = (uint32_t)(step0 + *step_base + (uint64_t)b / (uint64_t)per_step);
                blk = tn_philox(make_uint4((uint32_t)blk_id, (uint32_t)id, st, (inst << 2) | 0u), k0, k1);
            }
            const double ut = tn_u01(tn_word(blk, i & 3)) * tot;
            s = PD - 1;
            bool near = false;
#pragma unroll
            for (int q = PD - 1; q >= 0; --q)
                if (ut < cum[q]) s = q;   // the smallest q with u tot < cum_q
#pragma unroll
            for (int q = 0; q + 1 < PD; ++q) near |= fabs(ut - cum[q]) < 1e-6 * tot;
            if (j == 0) {
                row[c] = (int8_t)s;
                if (near) atomicAdd(&counters[CNT_NEAR], 1ull);
            }
        }
        double ws = w[0];
#pragma unroll
        for (int q = 1; q < PD; ++q)
            if (q == s) ws = w[q];
        lq += log(ws / tot);
        // energy: field, bond to the previous neighbour, bond above
        if (h) {
            double hs = hv[0];
#pragma unroll
            for (int q = 1; q < PD; ++q)
                if (q == s) hs = hv[q];
            E -= hs;
        }
        if (t > 0 && sprev == s) E -= jh;
        if (u == s) E -= jv;
        double nl = 0.0;
        if (pipe) {        // the drawn value's operands, loaded before the draw
#pragma unroll
            for (int a = 0; a < TP; ++a) {
                double ga = gd[0][a];
#pragma unroll
                for (int q = 1; q < PP; ++q)
                    if (q == s) ga = gd[q][a];
                nl += __shfl(lam, a, T) * ga;
            }
        } else if (D == T) {      // as in the sweep: a fixed T-term product
            const double *Gs = (rightward ? Gr : Gc) + ((size_t)c * PD + s) * DD;
#pragma unroll
            for (int a = 0; a < T; ++a) nl += __shfl(lam, a, T) * Gs[a * D + j];
        } else if (rightward) {   // Lam <- Lam G_c(s)
            const double *Gs = Gr + ((size_t)c * PD + s) * DD;
            for (int a = 0; a < Dl; ++a) {
                const double x = __shfl(lam, a, T);
                if (j < Dr) nl += x * Gs[a * D + j];
            }
        } else {           // Lam <- G_c(s) Lam
            const double *Gs = Gc + ((size_t)c * PD + s) * DD;
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

template <int T, int PD>
int launch_potts_rows(tn_ctx *ctx, int B, int8_t *S, bool eval, double *logq, double *energy, double *g,
                      uint64_t seed, uint64_t step0, int per_step, uint64_t first_id) {
    const int threads = 256;
    const size_t total = (size_t)B * T;
    const int blocks = (int)((total + threads - 1) / threads);
    const size_t DD = (size_t)ctx->D * ctx->D;
    const double *Gr = ctx->pG, *Gc = ctx->pG + (size_t)ctx->Ly * ctx->Lx * PD * DD;
    for (int r = 0; r < ctx->Ly; ++r) {
        hipLaunchKernelGGL((k_potts_rows<T, PD>), dim3(blocks), dim3(threads), 0, ctx->stream, r, B, ctx->Lx,
                           ctx->Ly, ctx->D, ctx->Jh, ctx->Jv, ctx->h, ctx->pq, ctx->dims, Gr, Gc, S,
                           eval ? 1 : 0, logq, energy, g, (uint32_t)seed, (uint32_t)(seed >> 32), first_id,
                           step0, ctx->dstep, per_step, (uint32_t)ctx->inst, ctx->counters);
        TN_HIP(ctx, hipGetLastError());
    }
    return TN_OK;
}

template <int T>
int launch_potts_d(tn_ctx *ctx, int B, int8_t *S, bool eval, double *logq, double *energy, double *g,
                   uint64_t seed, uint64_t step0, int per_step, uint64_t first_id) {
    switch (ctx->qd) {
    case 2: return launch_potts_rows<T, 2>(ctx, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 3: return launch_potts_rows<T, 3>(ctx, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 4: return launch_potts_rows<T, 4>(ctx, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 5: return launch_potts_rows<T, 5>(ctx, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 6: return launch_potts_rows<T, 6>(ctx, B, S, eval, logq, energy, g, seed, step0, per_step, first_id);
    default: return tn_fail(ctx, TN_EINVAL, "Potts d must be in 2..6");
    }
}

}  // namespace

int tn_run_potts(tn_ctx *ctx, int batch, uint64_t seed, uint64_t step0, int per_step, uint64_t first_id,
                 int8_t *states, bool eval, double *logq, double *energy, void *scr) {
    if (batch == 0) return TN_OK;
    if (per_step <= 0) return tn_fail(ctx, TN_EINVAL, "proposals per step must be positive");
    int rc;
    if (!scr) {
        if ((rc = tn_ensure(ctx, &ctx->gscr, &ctx->gscr_cap, tn_potts_scratch_bytes(ctx, batch)))) return rc;
        scr = ctx->gscr;
    }
    double *g = (double *)scr;
    int T = 1;
    while (T < ctx->D) T <<= 1;
    switch (T) {
    case 1: return launch_potts_d<1>(ctx, batch, states, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 2: return launch_potts_d<2>(ctx, batch, states, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 4: return launch_potts_d<4>(ctx, batch, states, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 8: return launch_potts_d<8>(ctx, batch, states, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 16: return launch_potts_d<16>(ctx, batch, states, eval, logq, energy, g, seed, step0, per_step, first_id);
    case 32: return launch_potts_d<32>(ctx, batch, states, eval, logq, energy, g, seed, step0, per_step, first_id);
    default: return tn_fail(ctx, TN_EINVAL, "Potts bond dimension above 32");
    }
}

extern "C" int tn_potts_build_env(tn_ctx *ctx, int Lx, int Ly, int d, const double *Jh, const double *Jv,
                                  const double *h, double beta, int D, double *logZ_out) {
    (void)hipGetLastError();
    if (!ctx) return TN_EINVAL;
    ctx->err.clear();
    if (ctx->capturing) return tn_fail(ctx, TN_ESTATE, "not allowed while capturing a graph");
    if (d < 2 || d > TN_POTTS_MAXD) return tn_fail(ctx, TN_EINVAL, "d must be in 2..6");
    if (Lx < 1 || Ly < 1) return tn_fail(ctx, TN_EINVAL, "Lx and Ly must be >= 1");
    if (Lx > 256) return tn_fail(ctx, TN_EINVAL, "Lx above 256 is not supported");
    if (D < 1 || D > TN_POTTS_MAXBOND) return tn_fail(ctx, TN_EINVAL, "D must be in 1..32 for Potts models");
    if (!std::isfinite(beta)) return tn_fail(ctx, TN_EINVAL, "beta must be finite");
    if (Lx > 1 && !Jh) return tn_fail(ctx, TN_EINVAL, "Jh is NULL");
    if (Ly > 1 && !Jv) return tn_fail(ctx, TN_EINVAL, "Jv is NULL");
    if (ctx->fit_sweeps) return tn_fail(ctx, TN_EINVAL, "Potts builds use successive SVD only (tn_set_compression 0)");
    ctx->building = false;
    ++ctx->env_gen;
    ctx->has_env = false;
    ctx->has_cst = false;
    ctx->qd = 0;
    const size_t nh = (size_t)Ly * (Lx - 1), nv = (size_t)(Ly - 1) * Lx, nf = (size_t)Ly * Lx * d;
    if (ctx->Jh) (void)hipFree(ctx->Jh);
    if (ctx->Jv) (void)hipFree(ctx->Jv);
    if (ctx->h) (void)hipFree(ctx->h);
    ctx->Jh = ctx->Jv = ctx->h = nullptr;
    TN_HIP(ctx, hipMalloc((void **)&ctx->Jh, (nh ? nh : 1) * sizeof(double)));
    TN_HIP(ctx, hipMalloc((void **)&ctx->Jv, (nv ? nv : 1) * sizeof(double)));
    if (nh) TN_HIP(ctx, hipMemcpyAsync(ctx->Jh, Jh, nh * sizeof(double), hipMemcpyDefault, ctx->stream));
    if (nv) TN_HIP(ctx, hipMemcpyAsync(ctx->Jv, Jv, nv * sizeof(double), hipMemcpyDefault, ctx->stream));
    if (h) {
        TN_HIP(ctx, hipMalloc((void **)&ctx->h, nf * sizeof(double)));
        TN_HIP(ctx, hipMemcpyAsync(ctx->h, h, nf * sizeof(double), hipMemcpyDefault, ctx->stream));
    }
    ctx->Lx = Lx;
    ctx->Ly = Ly;
    ctx->D = D;
    ctx->Dp = ((D + 15) / 16) * 16;
    ctx->beta = beta;
    ctx->prec = TN_FP64;
    int rc;
    const size_t ebox = (size_t)d * D * D;
    if ((rc = tn_ensure(ctx, (void **)&ctx->env, &ctx->env_cap, (size_t)(Ly + 1) * Lx * ebox * sizeof(double))))
        return rc;
    if (ctx->dims) (void)hipFree(ctx->dims);
    if (ctx->ell) (void)hipFree(ctx->ell);
    if (ctx->cst) (void)hipFree(ctx->cst);
    ctx->dims = nullptr;
    ctx->ell = nullptr;
    ctx->cst = nullptr;
    TN_HIP(ctx, hipMalloc((void **)&ctx->dims, (size_t)(Ly + 1) * (Lx + 1) * sizeof(int)));
    TN_HIP(ctx, hipMalloc((void **)&ctx->ell, (size_t)(Ly + 1) * sizeof(double)));
    TN_HIP(ctx, hipMalloc((void **)&ctx->cst, (size_t)(Ly + 1) * sizeof(int)));
    TN_HIP(ctx, hipMemsetAsync(ctx->ell, 0, (size_t)(Ly + 1) * sizeof(double), ctx->stream));
    TN_HIP(ctx, hipMemsetAsync(ctx->cst, 0xff, (size_t)(Ly + 1) * sizeof(int), ctx->stream));
    const PottsTab T(Lx, Ly, d);
    const PottsWork P(Lx, d, D);
    const size_t gsz = 2 * (size_t)Ly * Lx * d * D * D;
    if ((rc = tn_ensure(ctx, (void **)&ctx->pq, &ctx->pq_cap, T.total * sizeof(double)))) return rc;
    if ((rc = tn_ensure(ctx, (void **)&ctx->pw, &ctx->pw_cap, P.total * sizeof(double)))) return rc;
    if ((rc = tn_ensure(ctx, (void **)&ctx->pG, &ctx->pG_cap, gsz * sizeof(double)))) return rc;
    TN_HIP(ctx, hipMemsetAsync(ctx->counters + CNT_NOCONV, 0, sizeof(unsigned long long), ctx->stream));
    auto t0 = std::chrono::steady_clock::now();
    hipLaunchKernelGGL(k_potts_tab, dim3(64), dim3(256), 0, ctx->stream, Lx, Ly, d, beta, ctx->Jh, ctx->Jv,
                       ctx->h, ctx->pq);
    TN_HIP(ctx, hipGetLastError());
    // the trivial env below the last row: bond 1 everywhere
    std::vector<int> ones(Lx + 1, 1);
    TN_HIP(ctx, hipMemcpyAsync(ctx->dims + (size_t)Ly * (Lx + 1), ones.data(), (Lx + 1) * sizeof(int),
                               hipMemcpyHostToDevice, ctx->stream));
    for (int k = Ly - 1; k >= 1; --k) {
        hipLaunchKernelGGL(k_potts_row, dim3(1), dim3(256), 0, ctx->stream, k, Lx, Ly, d, D, ctx->pq, ctx->env,
                           ctx->dims, ctx->ell, ctx->pw, ctx->counters);
        TN_HIP(ctx, hipGetLastError());
    }
    hipLaunchKernelGGL(k_potts_top, dim3(1), dim3(256), 0, ctx->stream, Lx, Ly, d, D, ctx->pq, ctx->env,
                       ctx->dims, ctx->scal);
    TN_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL(k_potts_ops, dim3(1024), dim3(256), 0, ctx->stream, Lx, Ly, d, D, ctx->pq, ctx->env,
                       ctx->dims, ctx->pG, ctx->pG + gsz / 2);
    TN_HIP(ctx, hipGetLastError());
    double top[2];
    std::vector<double> ell(Ly + 1, 0.0);
    unsigned long long noconv = 0;
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));   // also keeps `ones` alive until its copy is done
    TN_HIP(ctx, hipMemcpy(top, ctx->scal, 2 * sizeof(double), hipMemcpyDeviceToHost));
    TN_HIP(ctx, hipMemcpy(ell.data(), ctx->ell, (Ly + 1) * sizeof(double), hipMemcpyDeviceToHost));
    TN_HIP(ctx, hipMemcpy(&noconv, ctx->counters + CNT_NOCONV, sizeof(noconv), hipMemcpyDeviceToHost));
    double lz = top[0];
    for (int k = 1; k < Ly; ++k) lz += ell[k];
    ctx->env_build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (noconv) return tn_fail(ctx, TN_ENOCONV, "Jacobi SVD did not converge in 60 sweeps");
    if (!(top[1] > 0.0) || !std::isfinite(lz))
        return tn_fail(ctx, TN_ENONPOS, "approximate partition function is not positive");
    ctx->logZ = lz;
    ctx->qd = d;
    ctx->has_env = true;
    if (logZ_out) *logZ_out = lz;
    return TN_OK;
}
