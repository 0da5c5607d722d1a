// Workgroup-level dense linear algebra shared by the environment build and
// the adjoint: Householder QR and the explicit Q factor, fp64, one workgroup
// (a multiple of 64 threads) operating on a matrix in LDS or global memory.
#pragma once

#include "common.hpp"

// Householder QR of A [m][n] (compact, ld = n) by one workgroup: R in the
// upper triangle, reflector j = (1, A[j+1:, j]) with coefficient tau[j].
static __device__ void wg_householder(double *A, int m, int n, double *tau) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int kk = min(m, n);
    for (int j = 0; j < kk; ++j) {
        if (w == 0) {
            double s2 = 0.0;
            for (int i = j + 1 + lane; i < m; i += 64) {
                const double x = A[i * n + j];
                s2 += x * x;
            }
            s2 = tn_wave_sum(s2);
            const double alpha = A[j * n + j];
            double t = 0.0, scl = 0.0, beta = alpha;
            if (s2 > 0.0) {
                beta = -copysign(sqrt(alpha * alpha + s2), alpha);
                t = (beta - alpha) / beta;
                scl = 1.0 / (alpha - beta);
            }
            for (int i = j + 1 + lane; i < m; i += 64) A[i * n + j] *= scl;
            if (lane == 0) {
                A[j * n + j] = beta;
                tau[j] = t;
            }
        }
        __syncthreads();
        const double t = tau[j];
        if (t != 0.0) {
            for (int l = j + 1 + w; l < n; l += nw) {
                double dot = 0.0;
                for (int i = j + lane; i < m; i += 64)
                    dot += (i == j ? 1.0 : A[i * n + j]) * A[i * n + l];
                dot = tn_wave_sum(dot);
                for (int i = j + lane; i < m; i += 64)
                    A[i * n + l] -= t * dot * (i == j ? 1.0 : A[i * n + j]);
            }
        }
        __syncthreads();
    }
}

// Q [m][kk] (ld ldq) = H_0 ... H_{kk-1} [I; 0] from the reflectors in A.
static __device__ void wg_form_q(const double *A, int m, int n, const double *tau, double *Q,
                          int ldq) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int kk = min(m, n);
    for (int t = threadIdx.x; t < m * kk; t += blockDim.x) {
        const int i = t / kk, l = t % kk;
        Q[i * ldq + l] = (i == l) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = kk - 1; j >= 0; --j) {
        const double tj = tau[j];
        if (tj != 0.0) {
            for (int l = j + w; l < kk; l += nw) {
                double dot = 0.0;
                for (int i = j + lane; i < m; i += 64)
                    dot += (i == j ? 1.0 : A[i * n + j]) * Q[i * ldq + l];
                dot = tn_wave_sum(dot);
                for (int i = j + lane; i < m; i += 64)
                    Q[i * ldq + l] -= tj * dot * (i == j ? 1.0 : A[i * n + j]);
            }
        }
        __syncthreads();
    }
}

