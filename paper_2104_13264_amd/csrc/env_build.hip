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
#include "linalg.hpp"

#include <chrono>
#include <cmath>
#include <vector>

namespace {

__global__ void k_fill_dims(int *dims, int n, int v) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
        dims[t] = v;
}

// X_c = sum_d env_{k+1,c}[a,d,b] M_{k,c}[l,u,d,x],  M = sum_s of the site
// tensor of App. A Eq. (tensor-general) with the field factor exp(beta h s).
__global__ void __launch_bounds__(256)
k_mpo_apply(int k, int Lx, int Ly, int D, double beta, const double *__restrict__ Jh,
            const double *__restrict__ Jv, const double *__restrict__ h,
            const double *__restrict__ env, const int *__restrict__ dims,
            double *__restrict__ xbox, int *__restrict__ xdims) {
    const int c = blockIdx.x;
    __shared__ double M[2][2][2][2];   // [l][u][d][x]
    const int lw = c > 0 ? 2 : 1, xw = c < Lx - 1 ? 2 : 1, dw = k < Ly - 1 ? 2 : 1;
    const bool triv = (k == Ly - 1);
    const int Dl = triv ? 1 : dims[(k + 1) * (Lx + 1) + c];
    const int Dr = triv ? 1 : dims[(k + 1) * (Lx + 1) + c + 1];
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
    double *X = xbox + (size_t)c * 8 * D * D;
    const int m = Dl * lw, n = Dr * xw, ld = 2 * D;
    const double *E = env + ((size_t)(k + 1) * Lx + c) * 2 * D * D;
    for (int t = threadIdx.x; t < m * 2 * n; t += blockDim.x) {
        const int j = t % n, rest = t / n, u = rest & 1, i = rest >> 1;
        const int a = i / lw, l = i % lw, b = j / xw, x = j % xw;
        double acc = 0.0;
        for (int d = 0; d < dw; ++d) {
            const double e = triv ? 1.0 : E[a * 2 * D + d * D + b];
            acc += e * M[l][u][d][x];
        }
        X[(i * 2 + u) * ld + j] = acc;
    }
    if (threadIdx.x == 0) {
        xdims[c] = m;
        xdims[Lx + 1 + c] = n;
    }
}

// One-sided (Hestenes) Jacobi on the rows of W [n][len]: plane rotations of
// row pairs, in the parallel round-robin order, until every pair is
// orthogonal to relative tolerance 4*len*eps; the same rotations are applied
// to the rows of Ut [n][n] (so that M = Ut^T W holds throughout).  Rows whose
// squared norm is below (len*eps)^2 ||W||_F^2 are numerically zero: they are
// not rotated and *zero2 receives that threshold so the caller drops them.
// Returns the number of sweeps, or -1 without convergence.
__device__ int wg_jacobi(double *W, double *Ut, int n, int len, int *flag, double *red,
                         double *zero2) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const double eps = 2.220446049250313e-16;
    double f2 = 0.0;
    for (int t = threadIdx.x; t < n * len; t += blockDim.x) f2 += W[t] * W[t];
    f2 = tn_block_sum(f2, red);
    const double small2 = f2 * (len * eps) * (len * eps);
    *zero2 = small2;
    if (n <= 1) return 0;
    const int npad = n + (n & 1);
    const double tol = 4.0 * len * eps;
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (threadIdx.x == 0) *flag = 0;
        __syncthreads();
        for (int t = 0; t < npad - 1; ++t) {
            for (int p = w; p < npad / 2; p += nw) {
                int i, j;
                if (p == 0) {
                    i = npad - 1;
                    j = t;
                } else {
                    i = (t + p) % (npad - 1);
                    j = (t - p + npad - 1) % (npad - 1);
                }
                if (i >= n || j >= n) continue;
                double a = 0.0, b = 0.0, g = 0.0;
                for (int e = lane; e < len; e += 64) {
                    const double x = W[i * len + e], y = W[j * len + e];
                    a += x * x;
                    b += y * y;
                    g += x * y;
                }
                a = tn_wave_sum(a);
                b = tn_wave_sum(b);
                g = tn_wave_sum(g);
                if (a > small2 && b > small2 && fabs(g) > tol * sqrt(a) * sqrt(b)) {
                    const double zeta = (b - a) / (2.0 * g);
                    const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
                    for (int e = lane; e < len; e += 64) {
                        const double x = W[i * len + e], y = W[j * len + e];
                        W[i * len + e] = cs * x - sn * y;
                        W[j * len + e] = sn * x + cs * y;
                    }
                    for (int e = lane; e < n; e += 64) {
                        const double x = Ut[i * n + e], y = Ut[j * n + e];
                        Ut[i * n + e] = cs * x - sn * y;
                        Ut[j * n + e] = sn * x + cs * y;
                    }
                    if (lane == 0) *flag = 1;
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

// Compress the MPO-MPS product of row k held in xbox and store env k.
// LDS layout (when it fits; else the same layout in global `gwork`):
//   B1 [8 D^2]  QR matrix / SVD matrix (first 4D^2) + SVD product (last 4D^2)
//   B2 [8 D^2]  explicit Q / R X product / U^T
__global__ void __launch_bounds__(1024)
k_truncate_row(int k, int Lx, int D, double *__restrict__ xbox, int *__restrict__ xdims,
               double *__restrict__ env, int *__restrict__ dims, double *__restrict__ ell,
               double *__restrict__ gwork, int use_lds,
               unsigned long long *__restrict__ counters, int *__restrict__ cst) {
    extern __shared__ double lds[];
    __shared__ double tau[2 * TN_MAX_D];
    __shared__ double sv[2 * TN_MAX_D];
    __shared__ int idx[2 * TN_MAX_D];
    __shared__ int mX[4 * TN_MAX_D + 1], nX[4 * TN_MAX_D + 1];
    __shared__ double red[16];
    __shared__ int flag;
    __shared__ double zero2;
    __shared__ int cmin;
    if (threadIdx.x == 0) cmin = -1;

    double *B1 = use_lds ? lds : gwork;
    double *B2 = B1 + 8 * D * D;
    const int ld = 2 * D;
    const size_t box = (size_t)8 * D * D;

    for (int c = threadIdx.x; c < Lx; c += blockDim.x) {
        mX[c] = xdims[c];
        nX[c] = xdims[Lx + 1 + c];
    }
    __syncthreads();

    // ---- left-to-right QR sweep: X_c <- Q, X_{c+1} <- R X_{c+1}
    for (int c = 0; c + 1 < Lx; ++c) {
        double *X = xbox + c * box, *Xn = xbox + (c + 1) * box;
        const int m = 2 * mX[c], n = nX[c], n1 = nX[c + 1];
        for (int t = threadIdx.x; t < m * n; t += blockDim.x) {
            const int r = t / n, j = t % n;
            B1[t] = X[r * ld + j];
        }
        __syncthreads();
        wg_householder(B1, m, n, tau);
        const int kk = min(m, n);
        wg_form_q(B1, m, n, tau, B2, kk);
        for (int t = threadIdx.x; t < m * kk; t += blockDim.x) {
            const int r = t / kk, p = t % kk;
            X[r * ld + p] = B2[t];
        }
        __syncthreads();
        // T[p][(u,j)] = sum_{q >= p} R[p][q] X_{c+1}[q][u][j]
        for (int t = threadIdx.x; t < kk * 2 * n1; t += blockDim.x) {
            const int p = t / (2 * n1), rem = t % (2 * n1), u = rem / n1, j = rem % n1;
            double acc = 0.0;
            for (int q = p; q < n; ++q) acc += B1[p * n + q] * Xn[(q * 2 + u) * ld + j];
            B2[t] = acc;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < kk * 2 * n1; t += blockDim.x) {
            const int p = t / (2 * n1), rem = t % (2 * n1), u = rem / n1, j = rem % n1;
            Xn[(p * 2 + u) * ld + j] = B2[t];
        }
        if (threadIdx.x == 0) {
            mX[c + 1] = kk;
            nX[c] = kk;
        }
        __syncthreads();
    }

    // ---- normalise the last column (its norm is the norm of the state)
    double lognorm;
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
        lognorm = log(nrm);
        __syncthreads();
    }

    // ---- right-to-left SVD sweep with truncation to D
    for (int c = Lx - 1; c >= 1; --c) {
        double *X = xbox + c * box, *Xp = xbox + (c - 1) * box;
        const int rows = mX[c], ncol = nX[c], len = 2 * ncol;
        double *W = B1, *T = B1 + 4 * D * D, *Ut = B2;
        for (int t = threadIdx.x; t < rows * len; t += blockDim.x) {
            const int i = t / len, e = t % len, u = e / ncol, j = e % ncol;
            W[t] = X[(i * 2 + u) * ld + j];
        }
        for (int t = threadIdx.x; t < rows * rows; t += blockDim.x)
            Ut[t] = (t / rows == t % rows) ? 1.0 : 0.0;
        __syncthreads();
        const int sweeps = wg_jacobi(W, Ut, rows, len, &flag, red, &zero2);
        if (sweeps < 0 && threadIdx.x == 0) atomicAdd(&counters[CNT_NOCONV], 1ull);
        {
            const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
            for (int i = w; i < rows; i += nw) {
                double s2 = 0.0;
                for (int e = lane; e < len; e += 64) s2 += W[i * len + e] * W[i * len + e];
                s2 = tn_wave_sum(s2);
                if (lane == 0) sv[i] = s2 > zero2 ? sqrt(s2) : 0.0;
            }
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
        // X_{c-1} <- X_{c-1} U[:, :chi] S[:chi]   (into T first)
        const int m1 = 2 * mX[c - 1];
        for (int t = threadIdx.x; t < m1 * chi; t += blockDim.x) {
            const int r = t / chi, kq = t % chi, ik = idx[kq];
            double acc = 0.0;
            for (int q = 0; q < rows; ++q) acc += Xp[r * ld + q] * Ut[ik * rows + q];
            T[t] = acc * sv[ik];
        }
        // X_c <- V^T[:chi]
        for (int t = threadIdx.x; t < chi * len; t += blockDim.x) {
            const int kq = t / len, e = t % len, u = e / ncol, j = e % ncol;
            const int ik = idx[kq];
            const double s = sv[ik];
            X[(kq * 2 + u) * ld + j] = s > 0.0 ? W[ik * len + e] / s : 0.0;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < m1 * chi; t += blockDim.x) {
            const int r = t / chi, kq = t % chi;
            Xp[r * ld + kq] = T[t];
        }
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
}

// ln <top|env_1>: row 0 (no up legs) contracted with env 1 left to right,
// rescaled by its largest entry after every column.  out[0] = ln|value|,
// out[1] = sign.
__global__ void __launch_bounds__(256)
k_top_overlap(int Lx, int Ly, int D, double beta, const double *__restrict__ Jh,
              const double *__restrict__ Jv, const double *__restrict__ h,
              const double *__restrict__ env, const int *__restrict__ dims,
              double *__restrict__ out) {
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

}  // namespace

int tn_top_overlap(tn_ctx *ctx, double *logtop, double *sign) {
    const int Lx = ctx->Lx, Ly = ctx->Ly, D = ctx->D;
    hipLaunchKernelGGL(k_top_overlap, dim3(1), dim3(256), 0, ctx->stream, Lx, Ly, D,
                       ctx->beta, ctx->Jh, ctx->Jv, ctx->h, ctx->env, ctx->dims, ctx->scal);
    TN_HIP(ctx, hipGetLastError());
    double hbuf[2];
    TN_HIP(ctx, hipMemcpyAsync(hbuf, ctx->scal, 2 * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *logtop = hbuf[0];
    *sign = hbuf[1];
    return TN_OK;
}

int tn_env_build_device(tn_ctx *ctx, double *logZ_out) {
    const int Lx = ctx->Lx, Ly = ctx->Ly, D = ctx->D;
    const size_t box = (size_t)8 * D * D;
    int rc;
    if ((rc = tn_ensure(ctx, (void **)&ctx->xbox, &ctx->xbox_cap, Lx * box * sizeof(double))))
        return rc;
    const bool use_lds = D <= 32;
    const size_t work = (size_t)16 * D * D;
    if (!use_lds &&
        (rc = tn_ensure(ctx, (void **)&ctx->wbuf, &ctx->wbuf_cap, work * sizeof(double))))
        return rc;
    if (!ctx->xdims) TN_HIP(ctx, hipMalloc((void **)&ctx->xdims, 2 * (4 * TN_MAX_D + 1) * sizeof(int) + 2 * 1024 * sizeof(int)));
    auto t0 = std::chrono::steady_clock::now();
    // trivial env below the last row: bond 1 everywhere
    hipLaunchKernelGGL(k_fill_dims, dim3(1), dim3(256), 0, ctx->stream,
                       ctx->dims + (size_t)Ly * (Lx + 1), Lx + 1, 1);
    TN_HIP(ctx, hipGetLastError());
    const size_t lds_bytes = use_lds ? work * sizeof(double) : 0;
    if (use_lds)
        TN_HIP(ctx, hipFuncSetAttribute((const void *)k_truncate_row,
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)lds_bytes));
    TN_HIP(ctx, hipMemsetAsync(ctx->counters + CNT_NOCONV, 0, sizeof(unsigned long long),
                               ctx->stream));
    for (int k = Ly - 1; k >= 1; --k) {
        hipLaunchKernelGGL(k_mpo_apply, dim3(Lx), dim3(256), 0, ctx->stream, k, Lx, Ly, D,
                           ctx->beta, ctx->Jh, ctx->Jv, ctx->h, ctx->env, ctx->dims,
                           ctx->xbox, ctx->xdims);
        TN_HIP(ctx, hipGetLastError());
        hipLaunchKernelGGL(k_truncate_row, dim3(1), dim3(1024), lds_bytes, ctx->stream, k, Lx,
                           D, ctx->xbox, ctx->xdims, ctx->env, ctx->dims, ctx->ell,
                           ctx->wbuf, use_lds ? 1 : 0, ctx->counters, ctx->cst);
        TN_HIP(ctx, hipGetLastError());
    }
    double logtop, sign;
    if ((rc = tn_top_overlap(ctx, &logtop, &sign))) return rc;
    std::vector<double> ell(Ly + 1, 0.0);
    TN_HIP(ctx, hipMemcpy(ell.data(), ctx->ell, (Ly + 1) * sizeof(double), hipMemcpyDeviceToHost));
    unsigned long long noconv = 0;
    TN_HIP(ctx, hipMemcpy(&noconv, ctx->counters + CNT_NOCONV, sizeof(noconv),
                          hipMemcpyDeviceToHost));
    auto t1 = std::chrono::steady_clock::now();
    ctx->env_build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    double lz = logtop;
    for (int k = 1; k < Ly; ++k) lz += ell[k];
    ctx->logZ = lz;
    if (logZ_out) *logZ_out = lz;
    if (noconv) return tn_fail(ctx, TN_ENOCONV, "Jacobi SVD did not converge in 60 sweeps");
    if (!(sign > 0.0) || !std::isfinite(lz))
        return tn_fail(ctx, TN_ENONPOS, "approximate partition function is not positive");
    return TN_OK;
}
