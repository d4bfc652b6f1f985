// Launch interface of the dense-coupling HMC kernels (dense_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "ihmc_internal.hpp"
#include "lattice_kernels.hpp"

namespace ihmc {

// K (FP64, N x N, row-major) -> three BF16 limbs and a zero-padded FP64 copy (Np x Np).
hipError_t dense_split_K(const double* K, int64_t N, int64_t Np, __bf16* Kl, double* K64, hipStream_t s);
// y = K x + C x in FP64 (padded length Np); a no-op once *stop is set (stop may be null).
hipError_t dense_gemv(const double* K64, int64_t Np, double C, const double* x, double* y, const int* stop,
                      hipStream_t s);
// h' = beta h (FP64) and h'/sqrt(J') (FP32) over the padded length.
hipError_t dense_field(const double* h, int64_t N, int64_t Np, double beta, double sqJ, double* hp, float* b,
                       hipStream_t s);
// Lanczos with full reorthogonalisation: normalised start vector, and step k
// (w = K q_k on entry; writes alpha[k], beta[k] and q_{k+1} = Q[k+1]).
constexpr int kLanczosMaxSteps = 1023;
hipError_t lanczos_start(double* q0, int64_t N, int64_t Np, hipStream_t s);
hipError_t lanczos_orth(double* Q, int k, double* w, double* alpha, double* beta, int64_t Np, hipStream_t s);
// Conjugate gradients on Kt (scal[0] = r.r, scal[1] = threshold; it[0] steps, it[1] stop flag).
hipError_t cg_init(const double* rhs, int64_t Np, double rel_tol, double* x, double* r, double* d, double* scal,
                   int* it, hipStream_t s);
hipError_t cg_step(const double* q, int64_t Np, double* x, double* r, double* d, double* scal, int* it,
                   hipStream_t s);
hipError_t dense_dot(const double* a, const double* b, int64_t Np, double* out, hipStream_t s);
hipError_t dense_fill(double* x, int64_t N, int64_t Np, double v, hipStream_t s);
// Split-K BF16-limb MFMA GEMM: part[s][b][i] over S slices of k; nprod = 3 or 6.
hipError_t dense_gemm_bf16(int nprod, const __bf16* Kl, const __bf16* Xl, float* part, int64_t Np, int64_t Bp, int S,
                           hipStream_t s);
// FP64 MFMA GEMM of K with the chains' stored fields (accepted field if measure,
// else the proposal after pass j).
hipError_t dense_gemm_f64(const double* K64, const ChainDev* chains, int j, int measure, double* U64, int64_t Np,
                          int B, hipStream_t s);
// Limbs of the accepted fields.
hipError_t dense_prep(const ChainDev* chains, int B, int64_t Np, int64_t Bp, __bf16* Xl, hipStream_t s);
// w = sqrt(J') tanh(sqrt(J') (K psi + C psi)) - psi for pass j.
hipError_t dense_epi_w(const ChainDev* chains, int B, int64_t Np, int64_t Bp, int S, const float* part, int j,
                       float* W32, __bf16* Wl, hipStream_t s);
// F = K w + C w + b, kick, drift (mode = FIRST / MIDDLE / LAST / FORCE).
hipError_t dense_epi_f(int mode, const ChainDev* chains, int B, int64_t Np, int64_t Bp, int S, const float* part,
                       const float* W32, int j, __bf16* Xl, hipStream_t s);
// FP64 action terms and the closing of each chain (mode = LAST or MEASURE).
hipError_t dense_h(int mode, const ChainDev* chains, int B, int64_t Np, const double* U64, int j, hipStream_t s);

}  // namespace ihmc
