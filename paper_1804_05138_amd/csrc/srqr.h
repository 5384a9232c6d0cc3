// Launchers of the spectrum-revealing swap steps (Alg. 3); see k_srqr.hip.
#pragma once

#include "internal.h"

namespace rq {

// Byte offsets of the SRQR scratch inside its part of the workspace.
struct SrqrLayout {
  size_t est, omega, part, cs, sc, iv, total;
  int nparts;
};
SrqrLayout srqr_layout(int m, int n, int l, int d, int exact);
// right-hand sides per workgroup of the triangular solve
int srqr_dw(int l1);

// est = trailing sketch norms^2 / lsk (positions l..n-1), 0 elsewhere.
int launch_srqr_init(hipStream_t s, int m, int n, int l, int lsk, double* a, long long lda,
                     int* jpvt, const double* b, long long ldb, double* est);
// pick (argmax est -> position l); if tau: Householder step on A(l:m, l:n),
// sc[0] = |R(l,l)|, sc[1] = tau.
int launch_srqr_pick_qr(hipStream_t s, int m, int n, int l, double* a, long long lda, int* jpvt,
                        double* est, double* tau, double* sc);
// g2 estimate (sc[2]) and the argmax row ii (iv[0]); om: d x (l+1) probe (ld d).
int launch_srqr_g2(hipStream_t s, int l, const double* a, long long lda, const double* om, int d,
                   int exact, const SrqrLayout& L, char* ws, double* g2_user);
// round robin of column iv[0] to position l and the Givens restoration.
int launch_srqr_rotate(hipStream_t s, int m, int n, int l, double* a, long long lda, int* jpvt,
                       const SrqrLayout& L, char* ws);

}  // namespace rq
