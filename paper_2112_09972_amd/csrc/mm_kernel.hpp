// Maffettone-Minale droplet model (arXiv 2112.09972, Sec. 2 Eqs. 1, 2, 5) for
// many trajectories at once: one thread per trajectory, FP64, classical RK4
// with `substeps` steps per row of the velocity-gradient table, A(t) linear
// between rows.  In the table's time unit the model reads
//   dM/dt = f2(Ca) (S M + M S) + W M - M W - (f1/tau_d) (M - 3 det(M)/II_M I),
// S, W the symmetric / antisymmetric parts of A, Ca = tau_d max|A_ij|,
// II_M = (tr(M)^2 - M:M)/2, f1, f2 of Eq. 5; tau_d = eta_s R / sigma.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sclbm {

struct Mat33 {
    double m[9];
};

__device__ __forceinline__ void mm_rhs(const double *M, const double *A, double tau_d, double chi, double *out) {
    double S[9], Wm[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            S[3 * i + j] = 0.5 * (A[3 * i + j] + A[3 * j + i]);
            Wm[3 * i + j] = 0.5 * (A[3 * i + j] - A[3 * j + i]);
        }
    double gmax = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) gmax = fmax(gmax, fabs(A[k]));
    const double ca = tau_d * gmax;
    const double f1 = 40.0 * (chi + 1.0) / ((3.0 + 2.0 * chi) * (16.0 + 19.0 * chi));
    const double f2 = 5.0 / (3.0 + 2.0 * chi) + 3.0 * ca * ca / (2.0 + 6.0 * ca * ca);
    const double tr = M[0] + M[4] + M[8];
    double mm = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) mm += M[k] * M[k];
    const double II = 0.5 * (tr * tr - mm);
    const double det = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                       M[2] * (M[3] * M[7] - M[4] * M[6]);
    const double c = 3.0 * det / II;
    const double relax = f1 / tau_d;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double sm = 0.0, ms = 0.0, wm = 0.0, mw = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                sm += S[3 * i + k] * M[3 * k + j];
                ms += M[3 * i + k] * S[3 * k + j];
                wm += Wm[3 * i + k] * M[3 * k + j];
                mw += M[3 * i + k] * Wm[3 * k + j];
            }
            out[3 * i + j] = f2 * (sm + ms) + wm - mw - relax * (M[3 * i + j] - (i == j ? c : 0.0));
        }
}

// A: [ntraj][nrows][9]; M0 (optional): [ntraj][9]; out: [ntraj][nrec][9] with
// nrec = 1 + (nrows - 1) / record_every, record r at time r * record_every.
__global__ __launch_bounds__(64) void k_mm(const double *A, int64_t ntraj, int64_t nrows, double tau_d, double chi,
                                           int substeps, int record_every, const double *M0, double *out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntraj) return;
    const double *At = A + t * nrows * 9;
    const int64_t nrec = 1 + (nrows - 1) / record_every;
    double *Ot = out + t * nrec * 9;
    double M[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) M[k] = M0 ? M0[t * 9 + k] : ((k % 4) == 0 ? 1.0 : 0.0);
#pragma unroll
    for (int k = 0; k < 9; ++k) Ot[k] = M[k];
    const double h = 1.0 / substeps;
    for (int64_t n = 0; n + 1 < nrows; ++n) {
        double A0[9], A1[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            A0[k] = At[n * 9 + k];
            A1[k] = At[(n + 1) * 9 + k];
        }
        for (int s = 0; s < substeps; ++s) {
            const double t0 = s * h;
            double Aa[9], Am[9], Ab[9], k1[9], k2[9], k3[9], k4[9], Y[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const double d = A1[k] - A0[k];
                Aa[k] = A0[k] + d * t0;
                Am[k] = A0[k] + d * (t0 + 0.5 * h);
                Ab[k] = A0[k] + d * (t0 + h);
            }
            mm_rhs(M, Aa, tau_d, chi, k1);
#pragma unroll
            for (int k = 0; k < 9; ++k) Y[k] = M[k] + 0.5 * h * k1[k];
            mm_rhs(Y, Am, tau_d, chi, k2);
#pragma unroll
            for (int k = 0; k < 9; ++k) Y[k] = M[k] + 0.5 * h * k2[k];
            mm_rhs(Y, Am, tau_d, chi, k3);
#pragma unroll
            for (int k = 0; k < 9; ++k) Y[k] = M[k] + h * k3[k];
            mm_rhs(Y, Ab, tau_d, chi, k4);
#pragma unroll
            for (int k = 0; k < 9; ++k) M[k] += (h / 6.0) * (k1[k] + 2.0 * k2[k] + 2.0 * k3[k] + k4[k]);
        }
        if ((n + 1) % record_every == 0) {
            const int64_t r = (n + 1) / record_every;
#pragma unroll
            for (int k = 0; k < 9; ++k) Ot[r * 9 + k] = M[k];
        }
    }
}

}  // namespace sclbm
