/*
 * ref_step.c - the FP64 oracle's explicit update in plain C.
 *
 * TEST INFRASTRUCTURE: part of the CPU oracle (see oracle/__init__.py); only
 * tests, the smoke check and the benchmark's CPU-baseline leg use it.  It
 * shares nothing with the GPU library.
 *
 * One step of the recurrence of Sec. V.A (Eq. 1 with the damping of
 * Listing 1, solved for u.forward; the adjoint of Listing 2 is the same
 * update run backwards in time):
 *
 *     out = A * u - B * up + C * (L_P u + extra / div)
 *
 * with L_P u[i] = sum_a sum_{k=-M..M} (c_|k| / h_a^2) u[i + k e_a] and u = 0
 * outside the array.  The terms are formed in exactly the order of the NumPy
 * oracle (oracle/fd.py laplacian, oracle/wave.py step), with no fused
 * multiply-adds (built with -ffp-contract=off), so both give the same bits.
 */
#include <stddef.h>
#include <stdint.h>

void awe_ref_step(const double* u, const double* up, double* out, const double* A, const double* B,
                  const double* C, const double* extra, double div, int ndim, const int64_t* n,
                  const double* coef /* [ndim][2M+1]: c_|k| / h_a^2 for k = -M..M */, int M) {
    const int64_t n0 = n[0], n1 = ndim >= 2 ? n[1] : 1, n2 = ndim >= 3 ? n[2] : 1;
    const int64_t s0 = n1 * n2, s1 = n2;
    const int K = 2 * M + 1;
#pragma omp parallel for schedule(static)
    for (int64_t i0 = 0; i0 < n0; ++i0) {
        for (int64_t i1 = 0; i1 < n1; ++i1) {
            for (int64_t i2 = 0; i2 < n2; ++i2) {
                const int64_t i = i0 * s0 + i1 * s1 + i2;
                double lap = 0.0;
                /* axis 0 */
                for (int k = -M; k <= M; ++k) {
                    const int64_t j = i0 + k;
                    const double v = (j >= 0 && j < n0) ? u[i + (int64_t)k * s0] : 0.0;
                    lap += coef[0 * K + (k + M)] * v;
                }
                if (ndim >= 2) {
                    for (int k = -M; k <= M; ++k) {
                        const int64_t j = i1 + k;
                        const double v = (j >= 0 && j < n1) ? u[i + (int64_t)k * s1] : 0.0;
                        lap += coef[1 * K + (k + M)] * v;
                    }
                }
                if (ndim >= 3) {
                    for (int k = -M; k <= M; ++k) {
                        const int64_t j = i2 + k;
                        const double v = (j >= 0 && j < n2) ? u[i + k] : 0.0;
                        lap += coef[2 * K + (k + M)] * v;
                    }
                }
                double rhs = lap;
                if (extra) rhs = lap + extra[i] / div;
                const double t1 = A[i] * u[i];
                const double t2 = B[i] * up[i];
                const double t3 = C[i] * rhs;
                out[i] = (t1 - t2) + t3;
            }
        }
    }
}
