// HMC with an explicit coupling matrix (Sec. 2: "replace the matrix JK by the
// full coupling matrix"; App. A's infinite-range model is one instance): the
// K~ products of the equations of motion become GEMMs over all chains at once,
//     U = K Psi + C Psi,   F = K W + C W + h'/sqrt(J'),  W = sqrt(J') tanh(sqrt(J') U) - Psi,
// with Psi the N x B matrix of the B chains' fields.
//
// Precision: K (FP64 input) is held as three BF16 limbs K = K0 + K1 + K2 and the
// FP32 operands Psi, W as three BF16 limbs as well (FP32 is exact in three).  A
// GEMM accumulates the limb products K_a X_b with a + b <= 2 (6 products;
// truncation ~2^-24 relative, i.e. FP32-accurate) or a + b <= 1 (3 products on
// two limbs, ~2^-16) in FP32 on the MFMA units.  C Psi and C W are added in FP32
// in the epilogues, so the diagonal never consumes BF16 precision.  The
// Hamiltonian uses an FP64 GEMM of the stored FP32 field with the FP64 K.
//
// Layouts:
//   K limbs   [L] x tiled (Np x Np), rows = sites i, columns = k
//   X limbs   [L] x tiled (Bp x Np), rows = chains b, columns = sites k
//   partials  [S][Bp][Np]  FP32 (split-K slices, summed in fixed order)
// "Tiled" stores each 128-row x 32-column block contiguously (8 KiB of BF16,
// rows of 64 bytes), blocks ordered row-block major: one k-step of a GEMM
// workgroup then reads one contiguous block per limb and operand, in whole
// cache lines.  Np is N padded to a multiple of 256, Bp is B padded to a
// multiple of 128; padding is zero.
#include "chain_epilogue.hpp"
#include "dense_kernels.hpp"
#include "device_common.hpp"

namespace ihmc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Offset of element (row, k) of a tiled operand with Np columns.
__host__ __device__ __forceinline__ int64_t tiled(int64_t row, int64_t k, int64_t Np) {
  return (((row >> 7) * (Np >> 5) + (k >> 5)) << 12) + ((row & 127) << 5) + (k & 31);
}
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Round-to-nearest-even BF16 limbs of a double: x ~ l0 + l1 + l2.
__device__ __forceinline__ void split3(double x, __bf16& l0, __bf16& l1, __bf16& l2) {
  l0 = (__bf16)(float)x;
  const double r1 = x - (double)(float)l0;
  l1 = (__bf16)(float)r1;
  const double r2 = r1 - (double)(float)l1;
  l2 = (__bf16)(float)r2;
}

// ------------------------------------------------------------ set-up kernels ---

// K (FP64, N x N) into limbs over the padded Np x Np layout; padding = 0.
__global__ void k_dense_split_K(const double* __restrict__ K, int64_t N, int64_t Np, __bf16* __restrict__ Kl) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= Np * Np) return;
  const int64_t i = idx / Np, k = idx % Np;
  const double x = (i < N && k < N) ? K[i * N + k] : 0.0;
  __bf16 a, b, c;
  split3(x, a, b, c);
  const int64_t o = tiled(i, k, Np);
  Kl[o] = a;
  Kl[Np * Np + o] = b;
  Kl[2 * Np * Np + o] = c;
}

// Padded FP64 copy of K for the Hamiltonian GEMM and the set-up solvers.
__global__ void k_dense_pad_K(const double* __restrict__ K, int64_t N, int64_t Np, double* __restrict__ K64) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= Np * Np) return;
  const int64_t i = idx / Np, k = idx % Np;
  K64[idx] = (i < N && k < N) ? K[i * N + k] : 0.0;
}

// y = K x + C x (FP64, one block of 256 threads per row; fixed-order reduction).
// A set `stop` flag turns the launch into a no-op (converged iterative solve).
__global__ __launch_bounds__(256) void k_dense_gemv(const double* __restrict__ K64, int64_t Np, double C,
                                                    const double* __restrict__ x, double* __restrict__ y,
                                                    const int* __restrict__ stop) {
  __shared__ double sh[4];
  if (stop && *stop) return;
  const int64_t i = blockIdx.x;
  const double* row = K64 + i * Np;
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < Np; k += 256) s += row[k] * x[k];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) y[i] = ((sh[0] + sh[1]) + (sh[2] + sh[3])) + C * x[i];
}

// Fixed-order sum over a 1024-thread block, broadcast to every thread.
__device__ double block_sum_1024(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < 16; ++w) t += sh[w];
  return t;
}

// Per-site field of a dense model: h' = beta h and h'/sqrt(J') (padding 0).
__global__ void k_dense_field(const double* __restrict__ h, int64_t N, int64_t Np, double beta, double sqJ,
                              double* __restrict__ hp, float* __restrict__ b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= Np) return;
  const double v = i < N ? beta * h[i] : 0.0;
  hp[i] = v;
  b[i] = (float)(v / sqJ);
}

// ---- Lanczos (lowest eigenvalue of K, for the shift C) ----------------------
//
// Start vector: normals of a fixed Philox stream, normalised (padding 0).
__global__ __launch_bounds__(1024) void k_lanczos_start(double* __restrict__ q0, int64_t N, int64_t Np) {
  __shared__ double sh[16];
  double ss = 0.0;
  for (int64_t i = threadIdx.x; i < Np; i += 1024) {
    double v = 0.0;
    if (i < N) {
      const uint4 r = philox4x32_10(make_uint4((uint32_t)(i >> 1), 0u, 0u, 0x4c414e43u), 0x2545f491u, 0x9e3779b9u);
      const double u1 = unit53(r.x, r.y), u2 = unit53(r.z, r.w);
      const double rad = sqrt(-2.0 * log(u1));
      v = (i & 1) ? rad * sin(2.0 * M_PI * u2) : rad * cos(2.0 * M_PI * u2);
    }
    q0[i] = v;
    ss += v * v;
  }
  ss = block_sum_1024(ss, sh);
  const double inv = 1.0 / sqrt(ss);
  for (int64_t i = threadIdx.x; i < Np; i += 1024) q0[i] *= inv;
}

// Step k of Lanczos with full reorthogonalisation (classical Gram-Schmidt,
// twice): w = K q_k on entry; alpha_k = q_k.w, w is orthogonalised against
// q_0..q_k, beta_k = |w|, q_{k+1} = w / beta_k.  One block of 1024 threads.
constexpr int kLanczosMax = 1024;
__global__ __launch_bounds__(1024) void k_lanczos_orth(double* __restrict__ Q, int k, double* __restrict__ w,
                                                       double* __restrict__ alpha, double* __restrict__ beta,
                                                       int64_t Np) {
  __shared__ double sc[kLanczosMax];
  __shared__ double sh[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double a = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int jj = wave; jj <= k; jj += 16) {
      const double* q = Q + (int64_t)jj * Np;
      double s = 0.0;
      for (int64_t i = lane; i < Np; i += 64) s += q[i] * w[i];
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) sc[jj] = s;
    }
    __syncthreads();
    a += sc[k];
    for (int64_t i = threadIdx.x; i < Np; i += 1024) {
      double s = 0.0;
      for (int jj = 0; jj <= k; ++jj) s += sc[jj] * Q[(int64_t)jj * Np + i];
      w[i] -= s;
    }
    __syncthreads();
  }
  double ss = 0.0;
  for (int64_t i = threadIdx.x; i < Np; i += 1024) ss += w[i] * w[i];
  ss = block_sum_1024(ss, sh);
  const double bk = sqrt(ss);
  const double inv = bk > 0.0 ? 1.0 / bk : 0.0;
  double* qn = Q + (int64_t)(k + 1) * Np;
  for (int64_t i = threadIdx.x; i < Np; i += 1024) qn[i] = w[i] * inv;
  if (threadIdx.x == 0) {
    alpha[k] = a;
    beta[k] = bk;
  }
}

// ---- conjugate gradients (Kt x = rhs, FP64) ---------------------------------
//
// scal[0] = r.r, scal[1] = stopping threshold, scal[2] = r.r at the start;
// it[0] counts iterations, it[1] is the stop flag read by the GEMV (1: converged,
// 2: a direction of non-positive curvature, i.e. Kt is not positive definite).
__global__ __launch_bounds__(1024) void k_cg_init(const double* __restrict__ rhs, int64_t Np, double rel_tol,
                                                  double* __restrict__ x, double* __restrict__ r,
                                                  double* __restrict__ d, double* __restrict__ scal,
                                                  int* __restrict__ it) {
  __shared__ double sh[16];
  double ss = 0.0;
  for (int64_t i = threadIdx.x; i < Np; i += 1024) {
    const double v = rhs[i];
    x[i] = 0.0;
    r[i] = v;
    d[i] = v;
    ss += v * v;
  }
  ss = block_sum_1024(ss, sh);
  if (threadIdx.x == 0) {
    scal[0] = ss;
    scal[1] = rel_tol * rel_tol * ss;
    scal[2] = ss;
    it[0] = 0;
    it[1] = (ss == 0.0) ? 1 : 0;
  }
}

__global__ __launch_bounds__(1024) void k_cg_step(const double* __restrict__ q, int64_t Np, double* __restrict__ x,
                                                  double* __restrict__ r, double* __restrict__ d,
                                                  double* __restrict__ scal, int* __restrict__ it) {
  __shared__ double sh[16];
  if (it[1]) return;
  const double rr = scal[0];
  double dq = 0.0;
  for (int64_t i = threadIdx.x; i < Np; i += 1024) dq += d[i] * q[i];
  dq = block_sum_1024(dq, sh);
  if (!(dq > 0.0)) {  // Kt not positive definite along d (or non-finite)
    if (threadIdx.x == 0) it[1] = 2;
    return;
  }
  const double alpha = rr / dq;
  double rn = 0.0;
  for (int64_t i = threadIdx.x; i < Np; i += 1024) {
    x[i] += alpha * d[i];
    r[i] -= alpha * q[i];
    rn += r[i] * r[i];
  }
  rn = block_sum_1024(rn, sh);
  const double bt = rn / rr;
  for (int64_t i = threadIdx.x; i < Np; i += 1024) d[i] = r[i] + bt * d[i];
  if (threadIdx.x == 0) {
    scal[0] = rn;
    it[0] += 1;
    if (!(rn > scal[1])) it[1] = 1;
  }
}

// out[0] = a.b (fixed order).
__global__ __launch_bounds__(1024) void k_dense_dot(const double* __restrict__ a, const double* __restrict__ b,
                                                    int64_t Np, double* __restrict__ out) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < Np; i += 1024) s += a[i] * b[i];
  s = block_sum_1024(s, sh);
  if (threadIdx.x == 0) out[0] = s;
}

__global__ void k_dense_fill(double* __restrict__ x, int64_t N, int64_t Np, double v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < Np) x[i] = i < N ? v : 0.0;
}

// ---------------------------------------------------------- split-K MFMA GEMM ---
//
// part[s][b][i] = sum_{k in slice s} sum_{(a, c) in products} Kl[a][i][k] * Xl[c][b][k]
// Workgroup tile 128 sites x 128 chains, k-step 32, eight waves (two per SIMD)
// of 32 sites x 64 chains (2 x 4 MFMA 16x16x32 tiles).  Operand tiles of all
// limbs are staged in LDS, double buffered: the global loads of k-step t+1 are
// issued into registers before the MFMAs of step t and written to the other
// LDS buffer after them, so one barrier per k-step separates the two.  LDS rows
// are padded to 40 elements, which makes the fragment reads conflict-free.
constexpr int GBM = 128, GBN = 128, GBK = 32, GPAD = 40, GTHREADS = 512;

template <int NL, int NPROD>
__global__ __launch_bounds__(GTHREADS) void k_dense_gemm_bf16(const __bf16* __restrict__ Kl,
                                                              const __bf16* __restrict__ Xl, float* __restrict__ part,
                                                              int64_t Np, int64_t Bp, int64_t kslice) {
  __shared__ __align__(16) __bf16 sA[2][NL][GBM][GPAD];
  __shared__ __align__(16) __bf16 sB[2][NL][GBN][GPAD];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * GBM, b0 = (int64_t)blockIdx.y * GBN;
  const int64_t k_begin = (int64_t)blockIdx.z * kslice;
  const int nk = (int)(kslice / GBK);
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 64;  // wave's sub-tile
  // limb pairs (a, c) with a + c <= 2 (NPROD = 6) or <= 1 (NPROD = 3)
  constexpr int PA[6] = {0, 0, 1, 0, 1, 2};
  constexpr int PC[6] = {0, 1, 0, 2, 1, 0};
  // staging: a 128 x 32 block is 512 chunks of 8 elements, contiguous in the
  // tiled layout; thread t moves chunk t (row t/4, k offset 8 (t%4)) per limb
  const int srow = t >> 2, skc = (t & 3) * 8;
  const __bf16* gA = Kl + tiled(i0, k_begin, Np) + t * 8;
  const __bf16* gB = Xl + tiled(b0, k_begin, Np) + t * 8;
  const int64_t lA = Np * Np, lB = Bp * Np;
  bf16x8 ra[NL], rb[NL];
  auto gload = [&](int64_t koff) {
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      ra[l] = *reinterpret_cast<const bf16x8*>(gA + l * lA + koff);
      rb[l] = *reinterpret_cast<const bf16x8*>(gB + l * lB + koff);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      *reinterpret_cast<bf16x8*>(&sA[buf][l][srow][skc]) = ra[l];
      *reinterpret_cast<bf16x8*>(&sB[buf][l][srow][skc]) = rb[l];
    }
  };

  f32x4 acc[2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};

  gload(0);
  lstore(0);
  lds_barrier();
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    // next 128 x 32 block of the same row block, issued before this step's MFMAs
    // and stored after them; unconditional (the last step reloads its own block
    // into the idle buffer), since the compiler sinks loads that only a branch
    // uses into that branch, after the MFMAs, exposing their whole latency
    gload((int64_t)min(kt + 1, nk - 1) << 12);
    __builtin_amdgcn_sched_barrier(0);
    bf16x8 fa[NL][2], fb[NL][4];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
#pragma unroll
      for (int r = 0; r < 2; ++r) fa[l][r] = *reinterpret_cast<const bf16x8*>(&sA[buf][l][wr + 16 * r + fr][fk]);
#pragma unroll
      for (int c = 0; c < 4; ++c) fb[l][c] = *reinterpret_cast<const bf16x8*>(&sB[buf][l][wc + 16 * c + fr][fk]);
    }
#pragma unroll
    for (int p = 0; p < NPROD; ++p)
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[PA[p]][r], fb[PC[p]][c], acc[r][c], 0, 0, 0);
    lstore(buf ^ 1);  // unconditional too, or the loads above would sink into its branch
    lds_barrier();
  }
  // D layout of the 16x16 MFMA: lane -> column (chain) lane % 16, rows 4 (lane / 16) + e
  float* out = part + (int64_t)blockIdx.z * Bp * Np;
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t b = b0 + wc + 16 * c + (lane & 15);
      const int64_t i = i0 + wr + 16 * r + 4 * (lane >> 4);
      *reinterpret_cast<float4*>(out + b * Np + i) = make_float4(acc[r][c][0], acc[r][c][1], acc[r][c][2], acc[r][c][3]);
    }
}

// ------------------------------------------------------------- FP64 MFMA GEMM ---
//
// U64[b][i] = sum_k K64[i][k] psi[b][k] with psi the stored FP32 fields (exact in
// FP64).  Tile 64 sites x 64 chains, k-step 32, four waves of 32 x 32 (2 x 2
// MFMA 16x16x4 FP64 tiles); LDS double buffered with register prefetch of the
// next k-step, as in the BF16 GEMM.
// The field of chain b is read through its state: the accepted field (with its
// sign) for a measurement, else the buffer holding the proposal after pass j.
constexpr int DBK = 32, DPAD = 33;

__global__ __launch_bounds__(256) void k_dense_gemm_f64(const double* __restrict__ K64,
                                                        const ChainDev* __restrict__ chains, int j, int measure,
                                                        double* __restrict__ U64, int64_t Np, int B) {
  __shared__ double sA[2][64][DPAD];
  __shared__ double sB[2][64][DPAD];
  __shared__ const float* sX[64];
  __shared__ float sS[64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int b0 = blockIdx.y * 64;
  if (t < 64) {
    const int b = b0 + t;
    const float* x = nullptr;
    float sg = 1.f;
    if (b < B) {
      const ChainDev& cd = chains[b];
      const ChainState* st = cd.st;
      const int buf = measure ? st->cur : pass_in_buf(st->cur, j);
      x = (const float*)cd.psi + (int64_t)buf * cd.NP;
      sg = (measure && st->sign < 0) ? -1.f : 1.f;
    }
    sX[t] = x;
    sS[t] = sg;
  }
  __syncthreads();
  // staging: A = 64 rows x 32 doubles as 1024 double2 chunks (4 per thread),
  // B = 64 rows x 32 floats as 512 float4 chunks (2 per thread)
  double2 ra[4];
  float4 rb[2];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ch = t + 256 * q, row = ch >> 4, c2 = (ch & 15) * 2;
      ra[q] = *reinterpret_cast<const double2*>(K64 + (i0 + row) * Np + k0 + c2);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int ch = t + 256 * q, row = ch >> 3, c4 = (ch & 7) * 4;
      const float* x = sX[row];
      rb[q] = x ? *reinterpret_cast<const float4*>(x + k0 + c4) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ch = t + 256 * q, row = ch >> 4, c2 = (ch & 15) * 2;
      sA[buf][row][c2] = ra[q].x;
      sA[buf][row][c2 + 1] = ra[q].y;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int ch = t + 256 * q, row = ch >> 3, c4 = (ch & 7) * 4;
      const float sg = sS[row];
      sB[buf][row][c4] = (double)(sg * rb[q].x);
      sB[buf][row][c4 + 1] = (double)(sg * rb[q].y);
      sB[buf][row][c4 + 2] = (double)(sg * rb[q].z);
      sB[buf][row][c4 + 3] = (double)(sg * rb[q].w);
    }
  };
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  f64x4 acc[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[r][c] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int nk = (int)(Np / DBK);
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((int64_t)(kt + 1) * DBK);
#pragma unroll
    for (int ks = 0; ks < DBK; ks += 4) {
      const int fr = lane & 15, fk = ks + (lane >> 4);
      double fa[2], fb[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) fa[r] = sA[buf][wr + 16 * r + fr][fk];
#pragma unroll
      for (int c = 0; c < 2; ++c) fb[c] = sB[buf][wc + 16 * c + fr][fk];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[r], fb[c], acc[r][c], 0, 0, 0);
    }
    if (kt + 1 < nk) lstore(buf ^ 1);
    lds_barrier();
  }
  // D layout of the FP64 16x16 MFMA: lane -> column lane % 16, rows lane / 16 + 4 e
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int b = b0 + wc + 16 * c + (lane & 15);
      if (b >= B) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = i0 + wr + 16 * r + (lane >> 4) + 4 * e;
        U64[(int64_t)b * Np + i] = acc[r][c][e];
      }
    }
}

// ---------------------------------------------------------------- epilogues ---

// Sum of the split-K partials in slice order.
// Three BF16 limbs of an FP32 value (exact: 3 x 8 significand bits cover 24).
__device__ __forceinline__ void split_f32(float x, __bf16& l0, __bf16& l1, __bf16& l2) {
  l0 = (__bf16)x;
  const float r1 = x - (float)l0;
  l1 = (__bf16)r1;
  l2 = (__bf16)(r1 - (float)l1);
}

// The per-site kernels below (set-up limbs, both force epilogues, the FP64 action
// terms) run one wave per tile of 256 sites of one chain (grid: tiles x chains,
// so the chain's fields are uniform loads) with four consecutive sites per lane:
// 16-byte loads and stores of the FP32 fields, 8-byte stores of the limbs (four
// consecutive sites are contiguous in the tiled layout), and one wave per CU
// slot instead of four, so that the whole grid is resident at once.  Sites past
// N (the padding up to Np) carry zeros.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
constexpr int EPI_SITES = 256, EPI_THREADS = 64;

__device__ __forceinline__ f32x4 ld_f4(const float* p) { return *reinterpret_cast<const f32x4*>(p); }
__device__ __forceinline__ void st_f4(float* p, f32x4 v) { *reinterpret_cast<f32x4*>(p) = v; }

__device__ __forceinline__ f32x4 sum_parts4(const float* __restrict__ part, int S, int64_t plane, int64_t off) {
  f32x4 s = ld_f4(part + off);
  for (int q = 1; q < S; ++q) s = s + ld_f4(part + (int64_t)q * plane + off);
  return s;
}

// limbs of four consecutive sites (row b, columns i .. i+3, i % 4 == 0)
__device__ __forceinline__ void store_limbs4(__bf16* __restrict__ X, int64_t limb_stride, int64_t b, int64_t i,
                                             int64_t Np, f32x4 v) {
  bf16x4 l0, l1, l2;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    __bf16 a, c, d;
    split_f32(v[e], a, c, d);
    l0[e] = a;
    l1[e] = c;
    l2[e] = d;
  }
  const int64_t o = tiled(b, i, Np);
  *reinterpret_cast<bf16x4*>(X + o) = l0;
  *reinterpret_cast<bf16x4*>(X + limb_stride + o) = l1;
  *reinterpret_cast<bf16x4*>(X + 2 * limb_stride + o) = l2;
}

// Start of a trajectory / set-up: limbs of the accepted fields (sign applied).
__global__ __launch_bounds__(EPI_THREADS) void k_dense_prep(const ChainDev* __restrict__ chains, int64_t Np,
                                                            int64_t Bp, __bf16* __restrict__ Xl) {
  const int b = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * EPI_SITES + 4 * threadIdx.x;
  const ChainDev& cd = chains[b];
  const ChainState* st = cd.st;
  f32x4 v = {0.f, 0.f, 0.f, 0.f};
  if (i < cd.N) {
    v = ld_f4((const float*)cd.psi + (int64_t)st->cur * cd.NP + i);
    if (st->sign < 0) v = -v;
  }
  store_limbs4(Xl, Bp * Np, b, i, Np, v);
}

// After U = K Psi: w = sqrt(J') tanh(sqrt(J') (U + C psi) + hw) - psi  -> W (FP32 and
// limbs); hw = h' in the shifted form (per site: sqrt(J') times the stored
// h'/sqrt(J')), else 0.
__global__ __launch_bounds__(EPI_THREADS) void k_dense_epi_w(const ChainDev* __restrict__ chains, int64_t Np,
                                                             int64_t Bp, int S, const float* __restrict__ part, int j,
                                                             float* __restrict__ W32, __bf16* __restrict__ Wl) {
  const int b = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * EPI_SITES + 4 * threadIdx.x;
  const ChainDev& cd = chains[b];
  const ChainState* st = cd.st;
  const int64_t o = (int64_t)b * Np + i;
  const f32x4 ku = sum_parts4(part, S, Bp * Np, o);
  f32x4 w = {0.f, 0.f, 0.f, 0.f};
  if (i < cd.N) {
    const int buf = (j == 0) ? st->cur : pass_in_buf(st->cur, j);
    f32x4 v = ld_f4((const float*)cd.psi + (int64_t)buf * cd.NP + i);
    if (j == 0 && st->sign < 0) v = -v;
    const float a = (float)cd.sqJ, C = (float)cd.C;
    f32x4 hw = {0.f, 0.f, 0.f, 0.f};
    if (cd.form == FORM_SHIFTED) {
      if (cd.h_kind == 2) {
        const f32x4 b4 = ld_f4((const float*)cd.b + i);
#pragma unroll
        for (int e = 0; e < 4; ++e) hw[e] = a * b4[e];
      } else {
        hw = f32x4{(float)cd.hw, (float)cd.hw, (float)cd.hw, (float)cd.hw};
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (i + e < cd.N) {
        const float u = __builtin_fmaf(C, v[e], ku[e]);
        w[e] = __builtin_fmaf(a, tanh_state(__builtin_fmaf(a, u, hw[e])), -v[e]);
      }
    }
  }
  st_f4(W32 + o, w);
  store_limbs4(Wl, Bp * Np, b, i, Np, w);
}

// After F = K W: F += C w + h'/sqrt(J'); kick p, drift psi (not on the last pass),
// new limbs of psi.  The FIRST pass draws the momenta (one Philox draw per pair
// of sites) and sums 1/2 p^2, the LAST pass sums 1/2 p^2 of the final momenta.
template <int MODE>
__global__ __launch_bounds__(EPI_THREADS) void k_dense_epi_f(const ChainDev* __restrict__ chains, int64_t Np,
                                                             int64_t Bp, int S, const float* __restrict__ part,
                                                             const float* __restrict__ W32, int j,
                                                             __bf16* __restrict__ Xl) {
  const int b = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * EPI_SITES + 4 * threadIdx.x;
  const ChainDev& cd = chains[b];
  ChainState* st = cd.st;
  const int64_t o = (int64_t)b * Np + i;
  const int cur = st->cur;
  double kick_d = 0.0, drift_d = 0.0;
  pass_coeffs(cd, j, kick_d, drift_d);
  const float kick = (MODE == PASS_FORCE) ? 1.f : (float)kick_d;
  const float drift = (float)drift_d;
  float* pmom = (float*)cd.p + i;
  const f32x4 kw = sum_parts4(part, S, Bp * Np, o);
  double kin[4] = {0.0, 0.0, 0.0, 0.0};
  f32x4 psi_new = {0.f, 0.f, 0.f, 0.f};
  if (i < cd.N) {
    const int in_buf = (MODE == PASS_FIRST || MODE == PASS_FORCE) ? cur : pass_in_buf(cur, j);
    f32x4 v = ld_f4((const float*)cd.psi + (int64_t)in_buf * cd.NP + i);
    if ((MODE == PASS_FIRST || MODE == PASS_FORCE) && st->sign < 0) v = -v;
    const f32x4 w = ld_f4(W32 + o);
    f32x4 bs = {0.f, 0.f, 0.f, 0.f};  // the shifted form has no linear term
    if (cd.form != FORM_SHIFTED) {
      if (cd.h_kind == 2) bs = ld_f4((const float*)cd.b + i);
      else bs = f32x4{(float)cd.b0, (float)cd.b0, (float)cd.b0, (float)cd.b0};
    }
    f32x4 p = {0.f, 0.f, 0.f, 0.f};
    if (MODE == PASS_FIRST) {
      if (cd.p_given) {
        p = ld_f4(pmom);
      } else {
        float z0, z1, z2, z3;
        normal_pair<float>(cd, (uint32_t)st->traj, TAG_MOM, i >> 1, z0, z1);
        normal_pair<float>(cd, (uint32_t)st->traj, TAG_MOM, (i >> 1) + 1, z2, z3);
        p = f32x4{z0, z1, z2, z3};
      }
    } else if (MODE != PASS_FORCE) {
      p = ld_f4(pmom);
    }
    f32x4 pn = {0.f, 0.f, 0.f, 0.f};
    const float C = (float)cd.C;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (i + e < cd.N) {
        const float F = __builtin_fmaf(C, w[e], kw[e]) + bs[e];
        pn[e] = __builtin_fmaf(kick, F, p[e]);
        if (MODE == PASS_FIRST) kin[e] = 0.5 * (double)p[e] * (double)p[e];
        if (MODE == PASS_LAST) kin[e] = 0.5 * (double)pn[e] * (double)pn[e];
        if (MODE == PASS_FIRST || MODE == PASS_MIDDLE) psi_new[e] = __builtin_fmaf(drift, pn[e], v[e]);
      }
    }
    if (MODE != PASS_LAST || cd.write_p_last) st_f4(pmom, pn);
    if (MODE == PASS_FIRST || MODE == PASS_MIDDLE)
      st_f4((float*)cd.psi + (int64_t)pass_out_buf(cur, j) * cd.NP + i, psi_new);
  }
  if (MODE == PASS_FIRST || MODE == PASS_MIDDLE) store_limbs4(Xl, Bp * Np, b, i, Np, psi_new);
  if (MODE == PASS_FIRST || MODE == PASS_LAST) {
    uint32_t bad = 0u;
    u128 acc[NTERM];
#pragma unroll
    for (int a = 0; a < NTERM; ++a) acc[a] = u128{0ull, 0ull};
    constexpr int a = (MODE == PASS_FIRST) ? T_K0 : T_K1;
    acc[a] = to_fixed(quad_sum(kin[0], kin[1], kin[2], kin[3]), bad);
    block_store_terms<1>(cd, acc, bad, a, a, MODE == PASS_FIRST ? CONTRIB_FIRST : CONTRIB_FINAL_KIN, blockIdx.x);
  }
}

// FP64 action terms of the proposal (LAST) or of the accepted field (MEASURE)
// from U64 = K psi; the block that finishes a chain last closes it (Metropolis
// or measurement).
template <int MODE>
__global__ __launch_bounds__(EPI_THREADS) void k_dense_h(const ChainDev* __restrict__ chains, int64_t Np,
                                                         const double* __restrict__ U64, int j) {
  const int b = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * EPI_SITES + 4 * threadIdx.x;
  const ChainDev& cd = chains[b];
  ChainState* st = cd.st;
  const int cur = st->cur;
  double h[4][4] = {};  // [term][site]
  if (i < cd.N) {
    const int buf = (MODE == PASS_MEASURE) ? cur : pass_in_buf(cur, j);
    f32x4 v4 = ld_f4((const float*)cd.psi + (int64_t)buf * cd.NP + i);
    if (MODE == PASS_MEASURE && st->sign < 0) v4 = -v4;
    const f64x4 ku = *reinterpret_cast<const f64x4*>(U64 + (int64_t)b * Np + i);
    f64x4 hp4 = {cd.hp0, cd.hp0, cd.hp0, cd.hp0};
    if (cd.h_kind == 2) hp4 = *reinterpret_cast<const f64x4*>(cd.hp + i);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (i + e < cd.N) {
        const double v = (double)v4[e];
        const double u = ku[e] + cd.C * v;
        const double hpx = hp4[e];
        const bool shifted = cd.form == FORM_SHIFTED;
        // shifted form: y = sqrt(J') u + h', no linear term, h[3] = y tanh(y)
        const double y = __builtin_fma(cd.sqJ, u, shifted ? hpx : 0.0);
        double lc, th;
        logcosh_tanh(y, lc, th);
        const double bx = shifted ? 0.0 : ((cd.h_kind == 2) ? hpx / cd.sqJ : cd.b0);
        h[0][e] = 0.5 * v * u - v * bx - lc;
        h[1][e] = v;
        h[2][e] = v * hpx;
        h[3][e] = (shifted ? y : u) * th;
      }
    }
  }
  uint32_t bad = 0u;
  u128 acc[NTERM];
#pragma unroll
  for (int a = 0; a < NTERM; ++a) acc[a] = u128{0ull, 0ull};
#pragma unroll
  for (int a = 0; a < 4; ++a) acc[T_S + a] = to_fixed(quad_sum(h[a][0], h[a][1], h[a][2], h[a][3]), bad);
  // the final kinetic energy was stored by the last force epilogue
  block_store_terms<1>(cd, acc, bad, T_S, T_UT, CONTRIB_ACTION, blockIdx.x);
  block_close<MODE == PASS_LAST, 1>(cd, st, MODE == PASS_LAST ? pass_in_buf(cur, j) : cur, blockIdx.x);
}

// ------------------------------------------------------------------ launch ---

hipError_t dense_split_K(const double* K, int64_t N, int64_t Np, __bf16* Kl, double* K64, hipStream_t s) {
  const int64_t n = Np * Np;
  const unsigned g = (unsigned)((n + 255) / 256);
  k_dense_split_K<<<g, 256, 0, s>>>(K, N, Np, Kl);
  k_dense_pad_K<<<g, 256, 0, s>>>(K, N, Np, K64);
  return hipGetLastError();
}

hipError_t dense_gemv(const double* K64, int64_t Np, double C, const double* x, double* y, const int* stop,
                      hipStream_t s) {
  k_dense_gemv<<<(unsigned)Np, 256, 0, s>>>(K64, Np, C, x, y, stop);
  return hipGetLastError();
}

hipError_t dense_field(const double* h, int64_t N, int64_t Np, double beta, double sqJ, double* hp, float* b,
                       hipStream_t s) {
  k_dense_field<<<(unsigned)((Np + 255) / 256), 256, 0, s>>>(h, N, Np, beta, sqJ, hp, b);
  return hipGetLastError();
}

hipError_t lanczos_start(double* q0, int64_t N, int64_t Np, hipStream_t s) {
  k_lanczos_start<<<1, 1024, 0, s>>>(q0, N, Np);
  return hipGetLastError();
}

hipError_t lanczos_orth(double* Q, int k, double* w, double* alpha, double* beta, int64_t Np, hipStream_t s) {
  if (k < 0 || k >= kLanczosMax) return hipErrorInvalidValue;
  k_lanczos_orth<<<1, 1024, 0, s>>>(Q, k, w, alpha, beta, Np);
  return hipGetLastError();
}

hipError_t cg_init(const double* rhs, int64_t Np, double rel_tol, double* x, double* r, double* d, double* scal,
                   int* it, hipStream_t s) {
  k_cg_init<<<1, 1024, 0, s>>>(rhs, Np, rel_tol, x, r, d, scal, it);
  return hipGetLastError();
}

hipError_t cg_step(const double* q, int64_t Np, double* x, double* r, double* d, double* scal, int* it,
                   hipStream_t s) {
  k_cg_step<<<1, 1024, 0, s>>>(q, Np, x, r, d, scal, it);
  return hipGetLastError();
}

hipError_t dense_dot(const double* a, const double* b, int64_t Np, double* out, hipStream_t s) {
  k_dense_dot<<<1, 1024, 0, s>>>(a, b, Np, out);
  return hipGetLastError();
}

hipError_t dense_fill(double* x, int64_t N, int64_t Np, double v, hipStream_t s) {
  k_dense_fill<<<(unsigned)((Np + 255) / 256), 256, 0, s>>>(x, N, Np, v);
  return hipGetLastError();
}

hipError_t dense_gemm_bf16(int nprod, const __bf16* Kl, const __bf16* Xl, float* part, int64_t Np, int64_t Bp, int S,
                           hipStream_t s) {
  dim3 grid((unsigned)(Np / GBM), (unsigned)(Bp / GBN), (unsigned)S);
  const int64_t kslice = Np / S;
  if (nprod == 6) k_dense_gemm_bf16<3, 6><<<grid, GTHREADS, 0, s>>>(Kl, Xl, part, Np, Bp, kslice);
  else k_dense_gemm_bf16<2, 3><<<grid, GTHREADS, 0, s>>>(Kl, Xl, part, Np, Bp, kslice);
  return hipGetLastError();
}

hipError_t dense_gemm_f64(const double* K64, const ChainDev* chains, int j, int measure, double* U64, int64_t Np,
                          int B, hipStream_t s) {
  dim3 grid((unsigned)(Np / 64), (unsigned)((B + 63) / 64));
  k_dense_gemm_f64<<<grid, 256, 0, s>>>(K64, chains, j, measure, U64, Np, B);
  return hipGetLastError();
}

hipError_t dense_prep(const ChainDev* chains, int B, int64_t Np, int64_t Bp, __bf16* Xl, hipStream_t s) {
  if (Np % EPI_SITES != 0) return hipErrorInvalidValue;
  k_dense_prep<<<dim3((unsigned)(Np / EPI_SITES), (unsigned)B), EPI_THREADS, 0, s>>>(chains, Np, Bp, Xl);
  return hipGetLastError();
}

hipError_t dense_epi_w(const ChainDev* chains, int B, int64_t Np, int64_t Bp, int S, const float* part, int j,
                       float* W32, __bf16* Wl, hipStream_t s) {
  if (Np % EPI_SITES != 0) return hipErrorInvalidValue;
  k_dense_epi_w<<<dim3((unsigned)(Np / EPI_SITES), (unsigned)B), EPI_THREADS, 0, s>>>(chains, Np, Bp, S, part, j,
                                                                                      W32, Wl);
  return hipGetLastError();
}

hipError_t dense_epi_f(int mode, const ChainDev* chains, int B, int64_t Np, int64_t Bp, int S, const float* part,
                       const float* W32, int j, __bf16* Xl, hipStream_t s) {
  if (Np % EPI_SITES != 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)(Np / EPI_SITES), (unsigned)B);
  switch (mode) {
    case PASS_FIRST:
      k_dense_epi_f<PASS_FIRST><<<grid, EPI_THREADS, 0, s>>>(chains, Np, Bp, S, part, W32, j, Xl);
      break;
    case PASS_MIDDLE:
      k_dense_epi_f<PASS_MIDDLE><<<grid, EPI_THREADS, 0, s>>>(chains, Np, Bp, S, part, W32, j, Xl);
      break;
    case PASS_LAST:
      k_dense_epi_f<PASS_LAST><<<grid, EPI_THREADS, 0, s>>>(chains, Np, Bp, S, part, W32, j, Xl);
      break;
    case PASS_FORCE:
      k_dense_epi_f<PASS_FORCE><<<grid, EPI_THREADS, 0, s>>>(chains, Np, Bp, S, part, W32, j, Xl);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t dense_h(int mode, const ChainDev* chains, int B, int64_t Np, const double* U64, int j, hipStream_t s) {
  if (Np % EPI_SITES != 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)(Np / EPI_SITES), (unsigned)B);
  if (mode == PASS_LAST) k_dense_h<PASS_LAST><<<grid, EPI_THREADS, 0, s>>>(chains, Np, U64, j);
  else k_dense_h<PASS_MEASURE><<<grid, EPI_THREADS, 0, s>>>(chains, Np, U64, j);
  return hipGetLastError();
}

}  // namespace ihmc
