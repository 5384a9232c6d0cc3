// Generic MFMA GEMM and explicit-Q helpers (see k_gemm.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace rq {

template <typename T>
int gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, T alpha, const T* A, long long lda,
         const T* B, long long ldb, T beta, T* C, long long ldc);

// Dense V (rows x bb), Gram V^T V and T of one reflector block.
template <typename T>
int block_t(hipStream_t s, int rows, int bb, const T* a, long long lda, const double* tau, T* vd,
            T* gram, T* tm);

size_t form_q_work_elems(int m, int k, int b);

template <typename T>
int form_q(hipStream_t s, int m, int k, int b, const T* a, long long lda, const double* tau, T* q,
           long long ldq, T* work);

}  // namespace rq
