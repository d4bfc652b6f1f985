// Fused leap-frog passes for HMC on periodic 2D / 3D nearest-neighbour lattices.
//
// One pass = one force evaluation of the equations of motion (Sec. 3):
//     u = Kt psi,  w = sqrt(J') tanh(sqrt(J') u) - psi,  F = Kt w + h'/sqrt(J'),
// followed by the kick p += c_j F and the drift psi' = psi + d_j p.  F at a
// site needs psi on the radius-2 diamond around it, so a workgroup stages psi
// on its tile plus a 2-wide halo in LDS, computes w on the tile plus a 1-wide
// halo, and then F, p and psi' on the tile: every pass reads psi, p (and the
// per-site field) once and writes p and psi' once.
//
// Pass kinds (template MODE):
//   FIRST   - momenta from Philox (Sec. 3, eq. momentum distribution), 1/2 p^2
//             accumulated for H_old, first kick and drift;
//   MIDDLE  - kick and drift;
//   LAST    - final kick, then the FP64 Hamiltonian and estimator sums of the
//             proposal; the block that finishes last takes the Metropolis
//             decision (Sec. 3) and writes the trajectory record;
//   MEASURE - FP64 action and estimator sums of the accepted field (set-up);
//   FORCE   - writes F itself (diagnostic; same arithmetic as the other passes).
// In 2D two MIDDLE steps can also run as one launch (lattice_pass2v_pair, the
// launch kind PASS_PAIR), with the per-site arithmetic of two passes.
//
// Memory layout: rows padded to `pitch` (a multiple of 4 elements), so a thread
// of the 2D kernel moves its four sites with 16-byte vector accesses.  Sums are
// exact 128-bit fixed point (device_common.hpp): results do not depend on the
// tile shape or on which chains share a launch.
#include "chain_epilogue.hpp"
#include "device_common.hpp"
#include "lattice_kernels.hpp"

namespace ihmc {

__device__ __forceinline__ int wrap_near(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }
// v mod L in [0, L) for |v| < 2^22 (lattice coordinates plus a halo): the
// quotient from FP32, exact to within one, then corrected in integers.
__device__ __forceinline__ int wrap_any(int v, int L) {
  const int q = (int)floorf((float)v * __builtin_amdgcn_rcpf((float)L));
  int r = v - q * L;
  r = r < 0 ? r + L : r;
  return r >= L ? r - L : r;
}

// The chain-state words a tiled pass reads at its start (accepted buffer,
// sign, trajectory index) do not change during the launch: only the block that
// closes the chain writes them, after every block of the launch has read them.
// They are read through the constant address space, so with scalar loads, and
// the buffer addresses derived from them stay in scalar registers.
__device__ __forceinline__ int32_t state_word(const int32_t* p) {
  return *(const __attribute__((address_space(4))) int32_t*)p;
}

template <typename T>
__device__ __forceinline__ T neg_if(T v, int sign) {
  return sign < 0 ? -v : v;
}

// Four consecutive state values (16 bytes for FP32, 32 bytes for FP64).
template <typename T>
__device__ __forceinline__ void ld4(const T* __restrict__ p, T (&v)[4]);
template <>
__device__ __forceinline__ void ld4<float>(const float* __restrict__ p, float (&v)[4]) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  v[0] = q.x;
  v[1] = q.y;
  v[2] = q.z;
  v[3] = q.w;
}
template <>
__device__ __forceinline__ void ld4<double>(const double* __restrict__ p, double (&v)[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0];
  const double2 b = reinterpret_cast<const double2*>(p)[1];
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}
// The state arrays that the chain table points to live in global memory.
// Accessing them through pointers of the global address space lets the
// compiler use global rather than flat memory instructions: a flat access
// counts as an LDS access too, so every wait for LDS data would also wait for
// the global loads still in flight.
template <class T>
using gmem = __attribute__((address_space(1))) T;
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ void ld4g(const gmem<T>* p, T (&v)[4]);
template <>
__device__ __forceinline__ void ld4g<float>(const gmem<float>* p, float (&v)[4]) {
  const vf4 q = *(const gmem<vf4>*)p;
  v[0] = q.x;
  v[1] = q.y;
  v[2] = q.z;
  v[3] = q.w;
}
template <>
__device__ __forceinline__ void ld4g<double>(const gmem<double>* p, double (&v)[4]) {
  const vd2 a = ((const gmem<vd2>*)p)[0];
  const vd2 b = ((const gmem<vd2>*)p)[1];
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}
template <typename T>
__device__ __forceinline__ void st4g(gmem<T>* p, const T (&v)[4]);
template <>
__device__ __forceinline__ void st4g<float>(gmem<float>* p, const float (&v)[4]) {
  *(gmem<vf4>*)p = vf4{v[0], v[1], v[2], v[3]};
}
template <>
__device__ __forceinline__ void st4g<double>(gmem<double>* p, const double (&v)[4]) {
  ((gmem<vd2>*)p)[0] = vd2{v[0], v[1]};
  ((gmem<vd2>*)p)[1] = vd2{v[2], v[3]};
}

// Where a staging thread finds its 4-element chunk x .. x+3 of every row it
// loads (x a multiple of 4, at least -4 and, when x_near, below 2 L0 - 4;
// x_near says every x + e lies within one period of [0, L0)): one aligned
// vector load at xv, or, for a chunk that straddles the periodic wrap, the
// four wrapped positions xe.  A wrapped chunk is still one vector load when L0
// is a multiple of 4.  Worked out once per thread, used for all its rows.
struct ChunkPos {
  int xv;
  bool vec;
  int xe[4];
};
__device__ __forceinline__ ChunkPos chunk_pos(int x, int L0, bool x_near) {
  ChunkPos cp;
  const int xs = x_near ? wrap_near(x, L0) : x;
  cp.vec = xs >= 0 && xs + 4 <= L0 && (xs & 3) == 0;
  cp.xv = cp.vec ? xs : 0;
  int xe = x_near ? xs : wrap_any(x, L0);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    cp.xe[e] = xe;
    xe = (xe + 1 == L0) ? 0 : xe + 1;
  }
  return cp;
}

// Every lane issues the vector load (a gathering lane from the row start, and
// discards it), so that the compiler keeps it one 16-byte access.
template <typename T>
__device__ __forceinline__ void load_chunk(const gmem<T>* row, const ChunkPos& cp, T (&v)[4]) {
  ld4g<T>(row + cp.xv, v);
  if (!cp.vec) {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = row[cp.xe[e]];
  }
}

// Element offset of a row from its index and the row pitch (both non-negative).
__device__ __forceinline__ uint64_t row_offset(int idx, int64_t stride) {
  return (uint64_t)(uint32_t)idx * (uint64_t)stride;
}

template <typename T>
__device__ __forceinline__ void st4(T* __restrict__ p, const T (&v)[4]);
template <>
__device__ __forceinline__ void st4<float>(float* __restrict__ p, const float (&v)[4]) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
template <>
__device__ __forceinline__ void st4<double>(double* __restrict__ p, const double (&v)[4]) {
  reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
  reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
}

// FP64 action and estimator terms of one site of the stored field: the integer
// stencil weights are exact, C and sqrt(J') are the true FP64 constants.
//   h[0]  S-density   1/2 psi u - psi h'/sqrt(J') - log cosh(sqrt(J') u)
//   h[1]  psi
//   h[2]  psi h'
//   h[3]  u tanh(sqrt(J') u)
// or, in the shifted form (b0 = 0, hw = h'), with y = sqrt(J') u + h':
//   h[0] = 1/2 psi u - log cosh(y),  h[3] = y tanh(y).
// `act` = the site belongs to the lattice (a quad may reach into the row
// padding, a column into the plane padding): inactive sites give exact zeros.
__device__ __forceinline__ void h_terms(const ChainDev& cd, double v, double nb, int64_t idx, bool act,
                                        double (&h)[4]) {
  const double u = cd.C * v + nb;
  const double y = __builtin_fma(cd.sqJ, u, cd.hw);
  double lc, th;
  logcosh_tanh(y, lc, th);
  double hpx = cd.hp0, bx = cd.b0;
  if (cd.h_kind == 2) {
    hpx = cd.hp[idx];
    bx = hpx / cd.sqJ;
  }
  h[0] = act ? 0.5 * v * u - v * bx - lc : 0.0;
  h[1] = act ? v : 0.0;
  h[2] = act ? v * hpx : 0.0;
  h[3] = act ? (cd.form == FORM_SHIFTED ? y : u) * th : 0.0;
}

// Workgroups are dealt to the eight XCDs round-robin (block b runs on XCD b % 8),
// each XCD with its own L2.  Neighbouring tiles read the same halo cache lines,
// so each XCD takes a contiguous range of the tile table: block b works on tile
// xcd_tile(b, n), a bijection of [0, n).
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int q = n >> 3, r = n & 7, k = b & 7, m = b >> 3;
  return k * q + (k < r ? k : r) + m;
}

// A LAST launch may cover chains whose trajectories end at different passes
// (j < 0): each block then takes its chain's own last pass j = n_pass - 1 and
// the launch index of that pass under the round's step plan (k != 0: the
// middle steps ran two per launch, so the last pass is launch j / 2 + 1;
// otherwise launch j).
__device__ __forceinline__ void chain_last_pass(const ChainDev& cd, int& j, int& k) {
  j = cd.n_pass - 1;
  k = k ? j / 2 + 1 : j;
}

// --------------------------------------------------------------------- 2D ---
//
// Tile BX x BY, one thread per quad of four consecutive x (NT = BX/4 * BY).
// LDS rows have pitch RP = BX + 8 with lattice x at index x - x0 + 4, so the
// psi halo [x0-2, x0+BX+2) sits inside one 16-byte aligned row and global and
// LDS traffic moves in aligned quads.  p and the per-site field are fetched
// after the staging, so their latency overlaps the barrier and the stencil
// work without holding up the staging.
template <typename T, int BX, int BY, int MODE>
__global__ __launch_bounds__(BX / 4 * BY) void lattice_pass2v(const ChainDev* __restrict__ chains,
                                                              const Tile* __restrict__ tiles, int n_tiles, int j,
                                                              int k) {
  constexpr int QX = BX / 4;
  constexpr int NT = QX * BY;
  constexpr int NWAVE = (NT + 63) / 64;
  constexpr int RP = BX + 8;
  constexpr int PR = BY + 4;
  constexpr int WR = BY + 2;
  constexpr int NWS = (BX + 2) * WR;
  constexpr int NCH = RP / 4;  // 16-byte chunks per staged row
  constexpr bool kHasW = (MODE != PASS_MEASURE);
  constexpr bool kH64 = (MODE == PASS_LAST || MODE == PASS_MEASURE);
  static_assert(BX % 4 == 0 && NT % 64 == 0, "tile shape");
  __shared__ __align__(16) T sP[PR * RP];
  __shared__ __align__(16) T sW[kHasW ? WR * RP : 4];

  const Tile tl = tiles[xcd_tile(blockIdx.x, n_tiles)];
  const ChainDev& cd = chains[tl.chain];
  ChainState* st = cd.st;
  const int L0 = cd.L0, L1 = cd.L1, pitch = cd.pitch;
  const int64_t NP = cd.NP;
  if (MODE == PASS_LAST && j < 0) chain_last_pass(cd, j, k);
  const int cur = state_word(&st->cur);
  const int sign = state_word(&st->sign);
  const int traj = state_word(&st->traj);
  const bool from_cur = (MODE == PASS_FIRST || MODE == PASS_MEASURE || MODE == PASS_FORCE);
  const int in_buf = from_cur ? cur : lat_in_buf(cur, k);
  const int out_buf = lat_out_buf(cur, k);
  const gmem<T>* __restrict__ pin = (const gmem<T>*)cd.psi + (int64_t)in_buf * NP;
  gmem<T>* __restrict__ pout = (gmem<T>*)cd.psi + (int64_t)out_buf * NP;
  // momenta: read from the buffer of launch k - 1, written to that of launch k
  // (the first, last and force passes use buffer 0)
  const gmem<T>* __restrict__ pmi = (const gmem<T>*)cd.p + (int64_t)lat_p_in(k) * NP;
  gmem<T>* __restrict__ pmo = (gmem<T>*)cd.p + (MODE == PASS_MIDDLE ? (int64_t)lat_p_out(k) * NP : 0);
  const bool site_field = (cd.h_kind == 2);

  const int t = threadIdx.x;
  const int qx = t % QX, qy = t / QX;
  const int gx = tl.x0 + 4 * qx, gy = tl.y0 + qy;
  const bool quad_ok = (gx < L0) && (gy < L1);  // the quad's first site is a lattice site
  const int64_t base = gx + (int64_t)pitch * gy;  // gx + 3 < pitch when quad_ok

  T pq[4] = {(T)0, (T)0, (T)0, (T)0};
  T bq[4];
  const T b_uniform = (T)cd.b0;
  bq[0] = bq[1] = bq[2] = bq[3] = b_uniform;

  // ---- stage psi on the tile plus its halo, in aligned 4-element chunks:
  // a chunk inside [0, L0) is one vector load, a chunk crossing the periodic
  // wrap (or the row end) is gathered element by element.
  // Thread t loads chunk column t % NCH of the rows t / NCH + RG k; all its
  // loads are issued before its LDS stores.
  const bool rows_near = (L1 > BY), x_near = (L0 > BX + 2);
  {
    constexpr int RG = NT / NCH;
    constexpr int NRPT = (PR + RG - 1) / RG;
    const int c = t % NCH, rg = t / NCH;
    if (rg < RG) {
      const ChunkPos cp = chunk_pos(tl.x0 - 4 + 4 * c, L0, x_near);
      T v[NRPT][4];
#pragma unroll
      for (int k = 0; k < NRPT; ++k) {
        const int r = rg + RG * k;
        if (r < PR) {
          const int yy = rows_near ? wrap_near(tl.y0 + r - 2, L1) : wrap_any(tl.y0 + r - 2, L1);
          load_chunk<T>(pin + row_offset(yy, pitch), cp, v[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < NRPT; ++k) {
        const int r = rg + RG * k;
        if (r < PR) {
          if (from_cur) {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[k][e] = neg_if(v[k][e], sign);
          }
          st4<T>(sP + r * RP + 4 * c, v[k]);
        }
      }
    }
  }
  // p and the field of the quad, issued after the staged rows' LDS stores
  // (loads complete in issue order: issued earlier, they would hold up the
  // wait for the staged values); their latency overlaps the barrier and w
  if (quad_ok) {
    if (MODE == PASS_MIDDLE || MODE == PASS_LAST || (MODE == PASS_FIRST && cd.p_given)) ld4g<T>(pmi + base, pq);
    if (kHasW && site_field) ld4g<T>((const gmem<T>*)cd.b + base, bq);
  }
  lds_barrier();

  const T Ct = (T)cd.C;
  const T at = (T)cd.sqJ, hw = (T)cd.hw;

  // ---- w on the rows y in [-1, BY], in quads over x in [-4, BX+4): the
  // outermost quads hold unused values (their stencil reaches past the staged
  // halo) but keep every LDS access aligned
  if (kHasW) {
    for (int i = t; i < WR * NCH; i += NT) {
      const int wy = i / NCH, c = i % NCH;
      const int pc = (wy + 1) * RP + 4 * c;  // psi at (x = -4 + 4c, y = wy - 1)
      T cv[4], up[4], dn[4], w[4];
      ld4<T>(sP + pc, cv);
      ld4<T>(sP + pc - RP, up);
      ld4<T>(sP + pc + RP, dn);
      const T lft = sP[pc - 1], rgt = sP[pc + 4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const T xm = (e == 0) ? lft : cv[e - 1];
        const T xp = (e == 3) ? rgt : cv[e + 1];
        const T s = (xm + xp) + (up[e] + dn[e]);
        const T u = fma_t(Ct, cv[e], s);
        w[e] = fma_t(at, tanh_state(fma_t(at, u, hw)), -cv[e]);
      }
      st4<T>(sW + wy * RP + 4 * c, w);
    }
    lds_barrier();
  }

  double kick_d = 0.0, drift_d = 0.0;
  pass_coeffs(cd, j, kick_d, drift_d);
  const T kick = (MODE == PASS_FORCE) ? (T)1 : (T)kick_d;
  const T drift = (T)drift_d;

  uint32_t bad = 0u;
  double qs[NTERM];  // FP64 sums of the thread's quad (0 without one)
#pragma unroll
  for (int a = 0; a < NTERM; ++a) qs[a] = 0.0;

  if (quad_ok) {
    // momenta of the first pass: one Philox draw per site pair; with an even
    // row length a pair never straddles a row
    if (MODE == PASS_FIRST && !cd.p_given) {
      const int64_t s0 = gx + (int64_t)L0 * gy;  // logical site of the quad's first element
      if ((L0 & 1) == 0) {
        normal_pair<T>(cd, (uint32_t)traj, TAG_MOM, s0 >> 1, pq[0], pq[1]);
        normal_pair<T>(cd, (uint32_t)traj, TAG_MOM, (s0 >> 1) + 1, pq[2], pq[3]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          T z0, z1;
          normal_pair<T>(cd, (uint32_t)traj, TAG_MOM, (s0 + e) >> 1, z0, z1);
          pq[e] = ((s0 + e) & 1) ? z1 : z0;
        }
      }
    }
    T pn[4], pv[4];
    const int pc0 = (qy + 2) * RP + 4 * qx + 4;  // psi of the quad's first site
    const int wc0 = (qy + 1) * RP + 4 * qx + 4;  // w of the quad's first site
    T cv[4];
    ld4<T>(sP + pc0, cv);
    T wcv[4], wup[4], wdn[4];
    if (kHasW) {
      ld4<T>(sW + wc0, wcv);
      ld4<T>(sW + wc0 - RP, wup);
      ld4<T>(sW + wc0 + RP, wdn);
    }
    double kin[4];
    double ht[4][4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const bool act = (gx + e < L0);
      const T c = cv[e];
      pv[e] = c;
      pn[e] = pq[e];
      kin[e] = 0.0;
      if (kHasW) {
        const T wm = (e == 0) ? sW[wc0 - 1] : wcv[e - 1];
        const T wp = (e == 3) ? sW[wc0 + 4] : wcv[e + 1];
        const T sw = (wm + wp) + (wup[e] + wdn[e]);
        const T F = fma_t(Ct, wcv[e], sw) + bq[e];
        pn[e] = fma_t(kick, F, (MODE == PASS_FORCE) ? (T)0 : pq[e]);
        pv[e] = fma_t(drift, pn[e], c);
        const double pd = (double)((MODE == PASS_FIRST) ? pq[e] : pn[e]);
        kin[e] = act ? 0.5 * pd * pd : 0.0;
      }
      if (kH64) {
        const int pc = pc0 + e;
        const double nb = ((double)sP[pc - 1] + (double)sP[pc + 1]) + ((double)sP[pc - RP] + (double)sP[pc + RP]);
        h_terms(cd, (double)c, nb, base + e, act, ht[e]);
      }
    }
    if (MODE == PASS_FIRST) qs[T_K0] = quad_sum(kin[0], kin[1], kin[2], kin[3]);
    if (MODE == PASS_LAST) qs[T_K1] = quad_sum(kin[0], kin[1], kin[2], kin[3]);
    if (kH64) {
#pragma unroll
      for (int a = 0; a < 4; ++a) qs[T_S + a] = quad_sum(ht[0][a], ht[1][a], ht[2][a], ht[3][a]);
    }
    if (MODE == PASS_FIRST || MODE == PASS_MIDDLE) {
      st4g<T>(pmo + base, pn);
      st4g<T>(pout + base, pv);
    } else if (MODE == PASS_FORCE || (MODE == PASS_LAST && cd.write_p_last)) {
      st4g<T>(pmo + base, pn);
    }
  }

  if (MODE == PASS_MIDDLE || MODE == PASS_FORCE) return;
  // Terms of 16 x-aligned sites: lanes 4m .. 4m+3 hold four consecutive quads
  // of one tile row (tile widths are multiples of 16), summed in FP64 as
  // (q0 + q1) + (q2 + q3) into every lane of the group; the group's lanes then
  // convert different terms to fixed point: the pass's terms T0 .. T0 + NU - 1
  // in rank order, rank 4r + j by lane j into accR[r].
  constexpr int T0 = (MODE == PASS_FIRST) ? T_K0 : ((MODE == PASS_MEASURE) ? T_S : T_K1);
  constexpr int NU = (MODE == PASS_FIRST) ? 1 : ((MODE == PASS_MEASURE) ? 4 : 5);
  constexpr int NR = (NU + 3) / 4;
  static_assert(QX % 4 == 0, "rows of whole 16-site groups");
  const int gl = threadIdx.x & 3;
  double gv[NU];
#pragma unroll
  for (int r = 0; r < NU; ++r) gv[r] = quad_sum_all(qs[T0 + r]);
  u128 accR[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    double x = 0.0;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
      if (4 * r + jj < NU) x = (gl == jj) ? gv[4 * r + jj] : x;
    accR[r] = to_fixed(x, bad);
  }
  const int tix = (tl.y0 / BY) * ((L0 + BX - 1) / BX) + tl.x0 / BX;  // tile index within the chain
  block_accumulate_ranks<MODE, NWAVE, NR>(cd, st, accR, bad, lat_in_buf(cur, k), tix);
}

// ------------------------------------------------------------ 2D, two steps ---
//
// Two consecutive middle leap-frog steps j, j + 1 in one pass over a tile.
// psi is staged with a 4-wide halo (rows y in [-4, BY+4), the x range of the
// one-step kernel); the first step's w is evaluated on the tile plus a 3-wide
// ring, its kick and drift on the tile plus a 2-wide ring, and the second
// step's w on a 1-wide ring and its kick and drift on the tile.  The first
// step on the ring repeats what the neighbouring tiles compute (about 15 %
// more arithmetic); in exchange the pair reads psi and p and writes them once,
// half the HBM traffic of two passes.  Per site the arithmetic is that of two
// MIDDLE passes, operation for operation, so the results are bit-identical.
//
// Positions outside the lattice (the ragged last tile of a row or column, the
// wrap of small lattices) hold periodic images: psi, p and the field are all
// loaded at wrapped coordinates, so every staged position evolves as the
// lattice site it images.  The ring's momenta are read from other tiles; they
// come from the buffer of launch k - 1 while the pair writes that of launch k,
// so no block reads momenta another block of the launch writes.
//
// A chain whose last middle step is step j (n_pass - 1 = j + 1) takes step j
// only: its blocks store the first step's tile results, which are those of the
// one-step pass, and skip the second.
//
// Threads work on quads of four consecutive x: TPQ = 1 gives each thread its
// tile quad (first-step momenta kept in registers for the second step) and at
// most one quad of the 2-wide ring (rows -2, -1, BY, BY+1 over the whole
// staged width, and the outer chunks of the tile rows); TPQ = 2 runs twice the
// threads, the first half on the tile quads and the second on the ring, so a
// launch of few tiles has more waves to hide latency with.

// w = sqrt(J') tanh(sqrt(J') u) - psi on the quad in chunk c of w-row wr, from
// psi in row wr + 1 of the staged rows (both arrays of pitch RP); the
// expression of the one-step kernel.
template <typename T, int RP>
__device__ __forceinline__ void pair_w_quad(const T* __restrict__ sP, T* __restrict__ sW, int wr, int c, T Ct,
                                            T at, T hw) {
  const int pc = (wr + 1) * RP + 4 * c;
  T cv[4], up[4], dn[4], w[4];
  ld4<T>(sP + pc, cv);
  ld4<T>(sP + pc - RP, up);
  ld4<T>(sP + pc + RP, dn);
  const T lft = sP[pc - 1], rgt = sP[pc + 4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const T xm = (e == 0) ? lft : cv[e - 1];
    const T xp = (e == 3) ? rgt : cv[e + 1];
    const T s = (xm + xp) + (up[e] + dn[e]);
    const T u = fma_t(Ct, cv[e], s);
    w[e] = fma_t(at, tanh_state(fma_t(at, u, hw)), -cv[e]);
  }
  st4<T>(sW + wr * RP + 4 * c, w);
}

// F = Kt w + h'/sqrt(J'), kick and drift of the quad in chunk c of w-row wr
// (psi in row wr + 1); the new field replaces psi in LDS.
template <typename T, int RP>
__device__ __forceinline__ void pair_kick_drift(T* __restrict__ sP, const T* __restrict__ sW, int wr, int c, T Ct,
                                                T kick, T drift, const T (&pq)[4], const T (&bq)[4], T (&pn)[4],
                                                T (&pv)[4]) {
  const int wc = wr * RP + 4 * c;
  const int pc = (wr + 1) * RP + 4 * c;
  T wcv[4], wup[4], wdn[4], cv[4];
  ld4<T>(sW + wc, wcv);
  ld4<T>(sW + wc - RP, wup);
  ld4<T>(sW + wc + RP, wdn);
  const T wl = sW[wc - 1], wrt = sW[wc + 4];
  ld4<T>(sP + pc, cv);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const T wm = (e == 0) ? wl : wcv[e - 1];
    const T wp = (e == 3) ? wrt : wcv[e + 1];
    const T sw = (wm + wp) + (wup[e] + wdn[e]);
    const T F = fma_t(Ct, wcv[e], sw) + bq[e];
    pn[e] = fma_t(kick, F, pq[e]);
    pv[e] = fma_t(drift, pn[e], cv[e]);
  }
  st4<T>(sP + pc, pv);
}

template <typename T, int BX, int BY, int TPQ>
__global__ __launch_bounds__(BX / 4 * BY * TPQ) void lattice_pass2v_pair(const ChainDev* __restrict__ chains,
                                                                         const Tile* __restrict__ tiles,
                                                                         int n_tiles, int j, int k) {
  constexpr int QX = BX / 4;
  constexpr int NQ = QX * BY;  // tile quads
  constexpr int NT = NQ * TPQ;
  constexpr int RP = BX + 8;  // staged x in [-4, BX+4)
  constexpr int NCH = RP / 4;
  constexpr int PR = BY + 8;  // psi rows y in [-4, BY+4)
  constexpr int WR = BY + 6;  // w rows y in [-3, BY+3)
  constexpr int NRING = 4 * NCH + 2 * BY;
  static_assert(BX % 4 == 0 && NQ % 64 == 0 && NRING <= NQ && (TPQ == 1 || TPQ == 2), "tile shape");
  __shared__ __align__(16) T sP[PR * RP];
  __shared__ __align__(16) T sW[WR * RP];

  const Tile tl = tiles[xcd_tile(blockIdx.x, n_tiles)];
  const ChainDev& cd = chains[tl.chain];
  const ChainState* st = cd.st;
  const int L0 = cd.L0, L1 = cd.L1, pitch = cd.pitch;
  const int64_t NP = cd.NP;
  const int cur = state_word(&st->cur);
  const gmem<T>* __restrict__ pin = (const gmem<T>*)cd.psi + (int64_t)lat_in_buf(cur, k) * NP;
  gmem<T>* __restrict__ pout = (gmem<T>*)cd.psi + (int64_t)lat_out_buf(cur, k) * NP;
  const gmem<T>* __restrict__ pmi = (const gmem<T>*)cd.p + (int64_t)lat_p_in(k) * NP;
  gmem<T>* __restrict__ pmo = (gmem<T>*)cd.p + (int64_t)lat_p_out(k) * NP;
  const gmem<T>* __restrict__ bfield = (const gmem<T>*)cd.b;
  const bool site_field = (cd.h_kind == 2);
  // rows y0 - 4 .. y0 + BY + 3 lie within one period of [0, L1) when L1 > BY + 3
  const bool rows_near = (L1 > BY + 3), x_near = (L0 > BX + 2);
  const int y0 = tl.y0;
  auto lat_row = [&](int y) { return rows_near ? wrap_near(y0 + y, L1) : wrap_any(y0 + y, L1); };

  const int t = threadIdx.x;
  const bool has_quad = (TPQ == 1) || t < NQ;
  const int tq = t % NQ;
  const int qx = tq % QX, qy = tq / QX;
  const int gx = tl.x0 + 4 * qx, gy = y0 + qy;
  const bool quad_ok = has_quad && (gx < L0) && (gy < L1);

  // ---- the thread's ring quad: row ry of the tile frame, chunk rc of the staged width
  const int rt = (TPQ == 1) ? t : t - NQ;  // ring quad index
  const bool has_ring = rt >= 0 && rt < NRING;
  int ry = 0, rc = 0;
  if (has_ring && rt < 4 * NCH) {
    const int ri = rt / NCH;
    ry = ri < 2 ? ri - 2 : BY + ri - 2;
    rc = rt % NCH;
  } else if (has_ring) {
    const int r2 = rt - 4 * NCH;
    ry = r2 >> 1;
    rc = (r2 & 1) ? NCH - 1 : 0;
  }

  // ---- stage psi on the tile plus its 4-wide halo, as in the one-step kernel.
  // The momenta and field loads are issued after the staged rows' LDS stores:
  // loads complete in issue order, so issued before them they would hold up
  // the wait for the staged values; issued here, their latency overlaps the
  // barrier and the first w, and the kick is their first use
  constexpr int RG = NT / NCH;
  constexpr int NRPT = (PR + RG - 1) / RG;
  const int sc = t % NCH, srg = t / NCH;
  T v[NRPT][4];
  if (srg < RG) {
    const ChunkPos cp = chunk_pos(tl.x0 - 4 + 4 * sc, L0, x_near);
#pragma unroll
    for (int q = 0; q < NRPT; ++q) {
      const int r = srg + RG * q;
      if (r < PR) load_chunk<T>(pin + row_offset(lat_row(r - 4), pitch), cp, v[q]);
    }
#pragma unroll
    for (int q = 0; q < NRPT; ++q) {
      const int r = srg + RG * q;
      if (r < PR) st4<T>(sP + r * RP + 4 * sc, v[q]);
    }
  }
  // ---- momenta and field of both quads, first needed by the kick
  T pq[4], bq[4], pr[4], br[4];
  const T b_uniform = (T)cd.b0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    bq[e] = b_uniform;
    br[e] = b_uniform;
    pq[e] = (T)0;
    pr[e] = (T)0;
  }
  {
    if (has_quad) {
      const ChunkPos cq = chunk_pos(gx, L0, x_near);
      const uint64_t oq = row_offset(lat_row(qy), pitch);
      load_chunk<T>(pmi + oq, cq, pq);
      if (site_field) load_chunk<T>(bfield + oq, cq, bq);
    }
    if (has_ring) {
      const ChunkPos cr = chunk_pos(tl.x0 - 4 + 4 * rc, L0, x_near);
      const uint64_t orr = row_offset(lat_row(ry), pitch);
      load_chunk<T>(pmi + orr, cr, pr);
      if (site_field) load_chunk<T>(bfield + orr, cr, br);
    }
  }

  lds_barrier();

  const T Ct = (T)cd.C;
  const T at = (T)cd.sqJ, hw = (T)cd.hw;
  double kick_d = 0.0, drift_d = 0.0;
  pass_coeffs(cd, j, kick_d, drift_d);
  const T kick1 = (T)kick_d, drift1 = (T)drift_d;
  pass_coeffs(cd, j + 1, kick_d, drift_d);
  const T kick2 = (T)kick_d, drift2 = (T)drift_d;

  // ---- step j: w on the rows y in [-3, BY+3) (w-row y + 3), all chunks (the
  // outermost quad of each row holds an unused value)
  for (int i = t; i < WR * NCH; i += NT) pair_w_quad<T, RP>(sP, sW, i / NCH, i % NCH, Ct, at, hw);
  lds_barrier();
  // kick and drift on the tile (momenta kept) and on the ring; each thread
  // overwrites only the psi of its own quads, which no other thread reads now
  T pa[4], va[4];
  if (has_quad) pair_kick_drift<T, RP>(sP, sW, qy + 3, qx + 1, Ct, kick1, drift1, pq, bq, pa, va);
  if (cd.n_pass - 1 == j + 1) {
    // the chain's last middle step is step j: its results are those of the
    // one-step pass, stored to the same buffers, and the block ends here
    if (quad_ok) {
      const int64_t base = gx + (int64_t)pitch * gy;
      st4g<T>(pmo + base, pa);
      st4g<T>(pout + base, va);
    }
    return;
  }
  if (has_ring) {
    T pn[4], pv[4];
    pair_kick_drift<T, RP>(sP, sW, ry + 3, rc, Ct, kick1, drift1, pr, br, pn, pv);
  }
  lds_barrier();

  // ---- step j + 1: w on the rows y in [-1, BY+1), then kick and drift on the tile
  for (int i = t; i < (BY + 2) * NCH; i += NT) pair_w_quad<T, RP>(sP, sW, 2 + i / NCH, i % NCH, Ct, at, hw);
  lds_barrier();
  if (!has_quad) return;
  T pn[4], pv[4];
  pair_kick_drift<T, RP>(sP, sW, qy + 3, qx + 1, Ct, kick2, drift2, pa, bq, pn, pv);
  if (quad_ok) {
    const int64_t base = gx + (int64_t)pitch * gy;
    st4g<T>(pmo + base, pn);
    st4g<T>(pout + base, pv);
  }
}

// ------------------------------------------------------------ 3D, one phase ---
//
// A block owns a BX x BY x ZR box, one thread per x-y column and aligned
// 4-plane slab (256 threads per slab: the LDS a box stages allows four boxes
// per CU, so an 8-plane box runs eight waves rather than four, to hide the
// latency of a chain too small to fill the GPU).  psi on the box plus its
// 2-wide halo is staged in LDS in one phase, in aligned 4-element chunks (rows
// of RP = BX + 8 values with lattice x at x - x0 + 4, as in 2D), so every load
// of the block is in flight at once; w on the box plus its 1-wide halo follows
// in quads (the outermost quad of a row is unused), then each thread updates
// its column's slab plane by plane.  The momenta and field values of the slab
// are fetched before the staging.  Sums of the FP64 terms follow the same
// order as in every other tiling: per column over each 4-plane slab in z order,
// then per x-aligned quad of columns.
template <typename T, int BX, int BY, int ZR, int MODE>
__global__ __launch_bounds__(64 * ZR, 8) void lattice_pass3t(const ChainDev* __restrict__ chains,
                                                          const Tile* __restrict__ tiles, int n_tiles, int j,
                                                          int k) {
  constexpr int NT = 64 * ZR;  // 256 threads per 4-plane slab
  constexpr int RP = BX + 8;
  constexpr int NCH = RP / 4;  // 16-byte chunks per staged row
  constexpr int PR = BY + 4, PZ = ZR + 4;
  constexpr int WR = BY + 2, WZ = ZR + 2;
  constexpr int PPL = PR * RP, WPL = WR * RP;
  constexpr bool kHasW = (MODE != PASS_MEASURE);
  constexpr bool kH64 = (MODE == PASS_LAST || MODE == PASS_MEASURE);
  static_assert(BX * BY == 256 && BX % 4 == 0 && ZR % 4 == 0, "one column and slab per thread");
  __shared__ __align__(16) T sP[PZ * PPL];
  __shared__ __align__(16) T sW[kHasW ? WZ * WPL : 4];

  const Tile tl = tiles[xcd_tile(blockIdx.x, n_tiles)];
  const ChainDev& cd = chains[tl.chain];
  ChainState* st = cd.st;
  if (MODE == PASS_LAST && j < 0) chain_last_pass(cd, j, k);
  const int L0 = cd.L0, L1 = cd.L1, L2 = cd.L2, pitch = cd.pitch;
  const int64_t NP = cd.NP;
  const int64_t plane = (int64_t)pitch * L1;
  const int cur = state_word(&st->cur);
  const int sign = state_word(&st->sign);
  const int traj = state_word(&st->traj);
  const bool from_cur = (MODE == PASS_FIRST || MODE == PASS_MEASURE || MODE == PASS_FORCE);
  const int in_buf = from_cur ? cur : lat_in_buf(cur, k);
  const int out_buf = lat_out_buf(cur, k);
  const gmem<T>* __restrict__ pin = (const gmem<T>*)cd.psi + (int64_t)in_buf * NP;
  gmem<T>* __restrict__ pout = (gmem<T>*)cd.psi + (int64_t)out_buf * NP;
  gmem<T>* __restrict__ pmom = (gmem<T>*)cd.p;
  const int z_end = min(tl.z0 + ZR, L2);
  const T b_uniform = (T)cd.b0;
  const gmem<T>* __restrict__ bsite = (const gmem<T>*)cd.b;
  const bool site_field = (cd.h_kind == 2);

  // ---- the momenta and field values of the thread's column and slab (planes
  // kz0 .. kz0 + 3 of the box)
  const int kz0 = 4 * (threadIdx.x / 256);
  const int lx = threadIdx.x % BX, ly = (threadIdx.x % 256) / BX;
  const int gx = tl.x0 + lx, gy = tl.y0 + ly;
  const bool act = (gx < L0) && (gy < L1);
  const int64_t col = gx + (int64_t)pitch * gy;
  constexpr bool kLoadP = (MODE == PASS_MIDDLE || MODE == PASS_LAST || MODE == PASS_FIRST);
  const bool load_p = kLoadP && act && (MODE != PASS_FIRST || cd.p_given);
  const bool load_b = kHasW && act && site_field;
  T pcol[4], bcol[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    pcol[k] = (T)0;
    bcol[k] = b_uniform;
    if (tl.z0 + kz0 + k < z_end) {
      if (load_p) pcol[k] = pmom[col + plane * (tl.z0 + kz0 + k)];
      if (load_b) bcol[k] = bsite[col + plane * (tl.z0 + kz0 + k)];
    }
  }

  // ---- stage psi on the box plus its halo: thread t owns chunk column c of
  // staged row r (each of the NCH * PR pairs has NH threads) and loads it in a
  // run of consecutive planes, so the row's wrap and offset are worked out
  // once; all its loads are issued before its LDS stores
  const bool rows_near = (L1 > BY), planes_near = (L2 > ZR), x_near = (L0 > BX + 2);
  {
    constexpr int NPAIR = NCH * PR;
    constexpr int NH = NT / NPAIR;
    constexpr int NPP = (PZ + NH - 1) / NH;  // planes per thread
    static_assert(NH >= 1, "box row too long for one block");
    const int pair = threadIdx.x % NPAIR, h = threadIdx.x / NPAIR;
    const int c = pair % NCH, r = pair / NCH;
    const int pz0 = h * NPP;
    T v[NPP][4];
    if (h < NH) {
      const ChunkPos cp = chunk_pos(tl.x0 - 4 + 4 * c, L0, x_near);
      const int yy = rows_near ? wrap_near(tl.y0 + r - 2, L1) : wrap_any(tl.y0 + r - 2, L1);
      const gmem<T>* rowy = pin + row_offset(yy, pitch);
      int zz = planes_near ? wrap_near(tl.z0 + pz0 - 2, L2) : wrap_any(tl.z0 + pz0 - 2, L2);
#pragma unroll
      for (int k = 0; k < NPP; ++k) {
        if (pz0 + k < PZ) load_chunk<T>(rowy + row_offset(zz, plane), cp, v[k]);
        zz = (zz + 1 == L2) ? 0 : zz + 1;
      }
    }
    // momenta of the first pass while the loads are in flight: one Philox draw
    // per site pair.  With an even row length the pair of column x (even) is
    // (x, x + 1), held by the neighbouring lane; over two planes the even lane
    // draws the pair of plane k, the odd lane that of plane k + 1, and each
    // passes its partner the partner's value.
    if (MODE == PASS_FIRST && !cd.p_given && (L0 & 1) == 0) {
      const bool even = (gx & 1) == 0;
#pragma unroll
      for (int k = 0; k < 4; k += 2) {
        const int64_t z = tl.z0 + kz0 + k + (even ? 0 : 1);
        const int64_t site = (gx & ~1) + (int64_t)L0 * (gy + (int64_t)L1 * z);
        T z0, z1;
        normal_pair<T>(cd, (uint32_t)traj, TAG_MOM, site >> 1, z0, z1);
        const T other = __shfl_xor(even ? z1 : z0, 1, 64);
        pcol[k] = even ? z0 : other;
        pcol[k + 1] = even ? other : z1;
      }
    }
    if (h < NH) {
#pragma unroll
      for (int k = 0; k < NPP; ++k) {
        if (pz0 + k < PZ) {
          if (from_cur) {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[k][e] = neg_if(v[k][e], sign);
          }
          st4<T>(sP + (pz0 + k) * PPL + r * RP + 4 * c, v[k]);
        }
      }
    }
  }
  lds_barrier();

  const T Ct = (T)cd.C;
  const T at = (T)cd.sqJ, hw = (T)cd.hw;

  // ---- w on the box plus its 1-wide halo, in quads over x in [-4, BX+4):
  // thread t computes chunk column t % NCH of the w rows t / NCH + RG k
  if (kHasW) {
    constexpr int NWROW = WZ * WR;
    constexpr int RG = NT / NCH;
    constexpr int NIT = (NWROW + RG - 1) / RG;
    const int c = threadIdx.x % NCH, rg = threadIdx.x / NCH;
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int R = rg + RG * k;
      if (rg >= RG || R >= NWROW) break;
      const int wz = R / WR, wy = R - wz * WR;
      const int pc = (wz + 1) * PPL + (wy + 1) * RP + 4 * c;  // psi at (x0 - 4 + 4c, y0 - 1 + wy, z0 - 1 + wz)
      T cv[4], up[4], dn[4], zm[4], zp[4], w[4];
      ld4<T>(sP + pc, cv);
      ld4<T>(sP + pc - RP, up);
      ld4<T>(sP + pc + RP, dn);
      ld4<T>(sP + pc - PPL, zm);
      ld4<T>(sP + pc + PPL, zp);
      const T lft = sP[pc - 1], rgt = sP[pc + 4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const T xm = (e == 0) ? lft : cv[e - 1];
        const T xp = (e == 3) ? rgt : cv[e + 1];
        T sum = (xm + xp) + (up[e] + dn[e]);
        sum = sum + (zm[e] + zp[e]);
        const T u = fma_t(Ct, cv[e], sum);
        w[e] = fma_t(at, tanh_state(fma_t(at, u, hw)), -cv[e]);
      }
      st4<T>(sW + wz * WPL + wy * RP + 4 * c, w);
    }
    lds_barrier();
  }

  double kick_d = 0.0, drift_d = 0.0;
  pass_coeffs(cd, j, kick_d, drift_d);
  const T kick = (MODE == PASS_FORCE) ? (T)1 : (T)kick_d;
  const T drift = (T)drift_d;

  // FP64 terms are summed per column over each aligned 4-plane slab (in z
  // order), then per x-aligned quad of columns, and converted to fixed point
  // once per slab and quad: the same grouping for every box depth.  The quad's
  // four lanes hold the same sums and deal the conversions: the pass's terms
  // T0 .. T0 + NU - 1 in rank order, rank 4k + j converted by lane j into accR[k].
  static_assert(ZR % 4 == 0, "boxes are whole 4-plane slabs");
  constexpr bool kAcc = (MODE == PASS_FIRST || MODE == PASS_LAST || MODE == PASS_MEASURE);
  constexpr int T0 = (MODE == PASS_FIRST) ? T_K0 : ((MODE == PASS_MEASURE) ? T_S : T_K1);
  constexpr int NU = (MODE == PASS_FIRST) ? 1 : ((MODE == PASS_MEASURE) ? 4 : 5);
  constexpr int NR = (NU + 3) / 4;
  const int ql = threadIdx.x & 3;
  uint32_t bad = 0u;
  double hs[NTERM];
  u128 accR[NR];
#pragma unroll
  for (int a = 0; a < NTERM; ++a) hs[a] = 0.0;
#pragma unroll
  for (int r = 0; r < NR; ++r) accR[r] = u128{0ull, 0ull};

#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = kz0 + kk;  // plane of the box
    const int z = tl.z0 + k;
    if (z < z_end) {
      const int64_t idx = col + plane * z;
      const int c = (k + 2) * PPL + (ly + 2) * RP + lx + 4;
      const T v = sP[c];
      double kin = 0.0;
      if (kHasW && act) {
        const int q = (k + 1) * WPL + (ly + 1) * RP + lx + 4;
        T sw = (sW[q - 1] + sW[q + 1]) + (sW[q - RP] + sW[q + RP]);
        sw = sw + (sW[q - WPL] + sW[q + WPL]);
        T F = fma_t(Ct, sW[q], sw);
        F = F + bcol[kk];
        T p;
        if (MODE == PASS_FIRST) {
          if (cd.p_given || (L0 & 1) == 0) {
            p = pcol[kk];
          } else {
            const int64_t site = gx + (int64_t)L0 * (gy + (int64_t)L1 * z);
            T z0, z1;
            normal_pair<T>(cd, (uint32_t)traj, TAG_MOM, site >> 1, z0, z1);
            p = (site & 1) ? z1 : z0;
          }
          const double pd = (double)p;
          kin = 0.5 * pd * pd;
        } else if (MODE == PASS_FORCE) {
          p = (T)0;
        } else {
          p = pcol[kk];
        }
        const T pn = fma_t(kick, F, p);
        if (MODE == PASS_FIRST || MODE == PASS_MIDDLE) {
          pmom[idx] = pn;
          pout[idx] = fma_t(drift, pn, v);
        } else if (MODE == PASS_FORCE) {
          pmom[idx] = pn;
        } else if (MODE == PASS_LAST) {
          if (cd.write_p_last) pmom[idx] = pn;
          const double pd = (double)pn;
          kin = 0.5 * pd * pd;
        }
      }
      if (MODE == PASS_FIRST) hs[T_K0] = hs[T_K0] + kin;
      if (MODE == PASS_LAST) hs[T_K1] = hs[T_K1] + kin;
      if (kH64) {
        double ht[4];
        double nb = ((double)sP[c - 1] + (double)sP[c + 1]) + ((double)sP[c - RP] + (double)sP[c + RP]);
        nb = nb + ((double)sP[c - PPL] + (double)sP[c + PPL]);
        h_terms(cd, (double)v, nb, act ? idx : 0, act, ht);
#pragma unroll
        for (int a = 0; a < 4; ++a) hs[T_S + a] = hs[T_S + a] + ht[a];
      }
    }
    // end of a slab: every lane takes part (the quad sums shuffle across the wave)
    if (kAcc && (k & 3) == 3) {
      double qv[NU];
#pragma unroll
      for (int r = 0; r < NU; ++r) {
        qv[r] = quad_sum_all(hs[T0 + r]);
        hs[T0 + r] = 0.0;
      }
#pragma unroll
      for (int kr = 0; kr < NR; ++kr) {
        double x = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (4 * kr + j < NU) x = (ql == j) ? qv[4 * kr + j] : x;
        accR[kr] = add128(accR[kr], to_fixed(x, bad));
      }
    }
  }

  if (MODE == PASS_MIDDLE || MODE == PASS_FORCE) return;
  const int tix = ((tl.z0 / ZR) * ((L1 + BY - 1) / BY) + tl.y0 / BY) * ((L0 + BX - 1) / BX) + tl.x0 / BX;
  block_accumulate_ranks<MODE, NT / 64, NR>(cd, st, accR, bad, lat_in_buf(cur, k), tix);
}

// ---------------------------------------------------- LDS-resident chains ---
//
// One workgroup runs whole trajectories of one small chain (one Tile entry per
// chain names it) with the accepted field, the working field, the momenta, w
// and the per-site field held in LDS in logical site order: every pass of the
// trajectory, its FP64 sums and the Metropolis step in one launch, with no
// partial-sum table and no launch per pass.  The per-site arithmetic and the
// grouping of the FP64 sums (in 2D 16 x-aligned sites as four quads; in 3D
// x-aligned quads of columns, each column first summed over an aligned 4-plane
// slab, in z order) are those of the tiled passes, so a resident chain's
// trajectory is bit-identical to the tiled one.
// n_traj = 0 measures S and the estimator sums of the accepted field (the
// set-up pass) instead.
constexpr int RES_THREADS = 256;
// field arrays: under half of the 160 KiB LDS with the reduction scratch, so
// two chains share a CU; 64 x 64 FP32 chains fit (without a per-site field)
constexpr int RES_LDS_BYTES = 81408;

int resident_max_sites(int precision, bool site_field) { return RES_LDS_BYTES / ((site_field ? 5 : 4) * precision); }

// LDS a launch reserves beyond the kernel's own when it runs beside tiled
// passes: enough that a CU holds one resident chain instead of two, so the
// other half of the CU's LDS stays with the tiled blocks (as many of them fit
// there as without it).
constexpr int RES_SOLO_LDS_PAD = 1024;
static_assert(2 * (RES_LDS_BYTES + RES_SOLO_LDS_PAD) > 160 * 1024, "one resident chain per CU");

// Two workgroups per CU also need the registers of two waves per SIMD (at most
// 256 per lane): left to itself the compiler spends more on the Metropolis
// step and the FP64 draws, which run once per trajectory, and the CU then
// holds one chain.  The bound keeps two, at the price of a few spilled FP64
// constants reloaded at the trajectory's end.
template <typename T, int NDIM>
__global__ __launch_bounds__(RES_THREADS, 2) void lattice_resident(const ChainDev* __restrict__ chains,
                                                                const Tile* __restrict__ tiles, int n_traj) {
  __shared__ __align__(16) unsigned char lds[RES_LDS_BYTES];
  __shared__ u128 sRed[RES_THREADS / 64][NTERM];
  __shared__ uint32_t sBad[RES_THREADS / 64];
  __shared__ int sSign, sTraj;
  __shared__ uint32_t sFlags;
  const ChainDev& cd = chains[tiles[blockIdx.x].chain];
  ChainState* st = cd.st;
  const int L0 = cd.L0, L1 = cd.L1, L2 = (NDIM == 3) ? cd.L2 : 1;
  const int N = (int)cd.N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool site_field = (cd.h_kind == 2);
  T* sA = reinterpret_cast<T*>(lds);  // accepted field as stored (sign not applied)
  T* sP = sA + N;                     // working field
  T* sM = sP + N;                     // momenta
  T* sW = sM + N;                     // w
  T* sB = sW + N;                     // h'/sqrt(J') per site (site field only)
  const int pitch = cd.pitch, plane = L0 * L1;
  const int cur = st->cur;
  gmem<T>* __restrict__ gpsi = (gmem<T>*)cd.psi + (int64_t)cur * cd.NP;
  for (int i = tid; i < N; i += RES_THREADS) {
    const int64_t g = (i % L0) + (int64_t)pitch * (i / L0);
    sA[i] = gpsi[g];
    if (site_field) sB[i] = ((const gmem<T>*)cd.b)[g];
  }
  const T b_uniform = (T)cd.b0;
  const T Ct = (T)cd.C;
  const T at = (T)cd.sqJ, hw = (T)cd.hw;

  // periodic neighbours of logical site i = x + L0 (y + L1 z)
  struct Nb {
    int xm, xp, ym, yp, zm, zp;
  };
  auto nbrs = [&](int i, int x, int y, int z) {
    Nb n;
    n.xm = i + (x == 0 ? L0 - 1 : -1);
    n.xp = i + (x == L0 - 1 ? 1 - L0 : 1);
    n.ym = i + (y == 0 ? (L1 - 1) * L0 : -L0);
    n.yp = i + (y == L1 - 1 ? -(L1 - 1) * L0 : L0);
    n.zm = i, n.zp = i;
    if (NDIM == 3) {
      n.zm = i + (z == 0 ? (L2 - 1) * plane : -plane);
      n.zp = i + (z == L2 - 1 ? -(L2 - 1) * plane : plane);
    }
    return n;
  };
  // FP64 sums of per-site terms into fixed point, grouped as in the tiled
  // passes: per 16 x-aligned sites, as (q0 + q1) + (q2 + q3) of their quads
  // (2D); per quad of columns each summed over an aligned 4-plane slab (3D).
  // term(i, x, y, z, out) fills the K terms listed in `which`; sites past the
  // row end contribute zeros.
  constexpr int UQ = (NDIM == 2) ? 4 : 1;  // quads per unit
  const int nq = (L0 + 4 * UQ - 1) / (4 * UQ), ns = (NDIM == 3) ? (L2 + 3) / 4 : 1;
  const int n_units = nq * L1 * ns;
  auto unit_sums = [&](auto term, const int* which, int K, u128* acc, uint32_t& bad) {
    for (int u = tid; u < n_units; u += RES_THREADS) {
      const int q = u % nq, r = u / nq, y = r % L1, sl = r / L1;
      // unit total (q0 + q1) + (q2 + q3) over its quads, built as the quads come
      double first[5], total[5];
#pragma unroll 1
      for (int g = 0; g < UQ; ++g) {
        double col[5][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
#pragma unroll
          for (int a = 0; a < 5; ++a) col[a][e] = 0.0;
          const int x = 4 * (UQ * q + g) + e;
          if (x >= L0) continue;
          const int z0 = 4 * sl, z1 = (NDIM == 3) ? min(z0 + 4, L2) : 1;
          for (int z = z0; z < z1; ++z) {
            double v[5];
            term(x + L0 * (y + L1 * z), x, y, z, v);
            for (int a = 0; a < K; ++a) col[a][e] = col[a][e] + v[a];
          }
        }
#pragma unroll
        for (int a = 0; a < 5; ++a) {
          const double qv = quad_sum(col[a][0], col[a][1], col[a][2], col[a][3]);
          if (UQ == 1) {
            total[a] = qv;
          } else if ((g & 1) == 0) {
            first[a] = qv;
          } else {
            const double pr = first[a] + qv;
            total[a] = (g == 1) ? pr : total[a] + pr;
          }
        }
      }
      for (int a = 0; a < K; ++a) acc[which[a]] = add128(acc[which[a]], to_fixed(total[a], bad));
    }
  };
  // S-density, psi, psi h', u tanh(sqrt(J') u) of the field in sP (FP64)
  auto action_terms = [&](int i, int x, int y, int z, double* v) {
    const Nb n = nbrs(i, x, y, z);
    double nb = ((double)sP[n.xm] + (double)sP[n.xp]) + ((double)sP[n.ym] + (double)sP[n.yp]);
    if (NDIM == 3) nb = nb + ((double)sP[n.zm] + (double)sP[n.zp]);
    double h[4];
    h_terms(cd, (double)sP[i], nb, x + (int64_t)pitch * (y + (int64_t)L1 * z), true, h);
    v[0] = h[0];
    v[1] = h[1];
    v[2] = h[2];
    v[3] = h[3];
  };
  // the block's fixed-point totals, for thread 0
  auto block_total = [&](const u128* acc, uint32_t bad, u128* sum) {
#pragma unroll
    for (int a = 0; a < NTERM; ++a) {
      const u128 v = wave_sum128(acc[a]);
      if (lane == 0) sRed[wave][a] = v;
    }
    const unsigned long long any = __ballot(bad != 0u);
    if (lane == 0) sBad[wave] = any ? 1u : 0u;
    __syncthreads();
    uint32_t b = 0u;
    if (tid == 0) {
      for (int a = 0; a < NTERM; ++a) {
        u128 v = sRed[0][a];
        for (int w = 1; w < RES_THREADS / 64; ++w) v = add128(v, sRed[w][a]);
        sum[a] = v;
      }
      for (int w = 0; w < RES_THREADS / 64; ++w) b |= sBad[w];
    }
    return b;
  };
  // The sites of a thread are tid, tid + NTHR, ...: their coordinates start
  // from those of tid and advance by fixed steps with carries, which keeps
  // integer division out of the pass loops.
  struct Walk {
    int x, y, z;
  };
  const int step_x = RES_THREADS % L0, step_r = RES_THREADS / L0;
  const int step_y = step_r % L1, step_z = step_r / L1;
  Walk w0;
  w0.x = tid % L0;
  w0.y = (tid / L0) % L1;
  w0.z = (tid / L0) / L1;
  auto advance_walk = [&](Walk& c) {
    c.x += step_x;
    int carry = 0;
    if (c.x >= L0) {
      c.x -= L0;
      carry = 1;
    }
    c.y += step_y + carry;
    carry = 0;
    if (c.y >= L1) {
      c.y -= L1;
      carry = 1;
    }
    c.z += step_z + carry;
  };

  if (n_traj == 0) {  // set-up: S and the estimator sums of the accepted field
    const int sign = st->sign;
    for (int i = tid; i < N; i += RES_THREADS) sP[i] = neg_if(sA[i], sign);
    __syncthreads();
    u128 acc[NTERM];
    for (int a = 0; a < NTERM; ++a) acc[a] = u128{0ull, 0ull};
    uint32_t bad = 0u;
    const int which[4] = {T_S, T_PSI, T_PSIH, T_UT};
    unit_sums(action_terms, which, 4, acc, bad);
    u128 sum[NTERM];
    const uint32_t b = block_total(acc, bad, sum);
    if (tid == 0) finalize_measure(st, sum, b);
    return;
  }

  for (int t = 0; t < n_traj; ++t) {
    if (tid == 0) {
      sSign = st->sign;
      sTraj = st->traj;
    }
    __syncthreads();
    const int sign = sSign;
    const uint32_t traj = (uint32_t)sTraj;
    // working field; fresh momenta, one Philox draw per site pair
    for (int i = tid; i < N; i += RES_THREADS) sP[i] = neg_if(sA[i], sign);
    for (int pr = tid; 2 * pr < N; pr += RES_THREADS) {
      T z0, z1;
      normal_pair<T>(cd, traj, TAG_MOM, pr, z0, z1);
      sM[2 * pr] = z0;
      if (2 * pr + 1 < N) sM[2 * pr + 1] = z1;
    }
    __syncthreads();
    u128 acc[NTERM];
    for (int a = 0; a < NTERM; ++a) acc[a] = u128{0ull, 0ull};
    uint32_t bad = 0u;
    {
      const int which[1] = {T_K0};
      unit_sums([&](int i, int, int, int, double* v) {
        const double pd = (double)sM[i];
        v[0] = 0.5 * pd * pd;
      }, which, 1, acc, bad);
    }
    // kick-drift passes; the last one kicks only
    for (int j = 0; j < cd.n_pass; ++j) {
      Walk cw = w0;
      for (int i = tid; i < N; i += RES_THREADS, advance_walk(cw)) {
        const Nb n = nbrs(i, cw.x, cw.y, cw.z);
        const T c = sP[i];
        T s = (sP[n.xm] + sP[n.xp]) + (sP[n.ym] + sP[n.yp]);
        if (NDIM == 3) s = s + (sP[n.zm] + sP[n.zp]);
        const T u = fma_t(Ct, c, s);
        sW[i] = fma_t(at, tanh_state(fma_t(at, u, hw)), -c);
      }
      __syncthreads();
      double kick_d = 0.0, drift_d = 0.0;
      pass_coeffs(cd, j, kick_d, drift_d);
      const T kick = (T)kick_d, drift = (T)drift_d;
      const bool last = (j == cd.n_pass - 1);
      Walk cu = w0;
      for (int i = tid; i < N; i += RES_THREADS, advance_walk(cu)) {
        const Nb n = nbrs(i, cu.x, cu.y, cu.z);
        T sw = (sW[n.xm] + sW[n.xp]) + (sW[n.ym] + sW[n.yp]);
        if (NDIM == 3) sw = sw + (sW[n.zm] + sW[n.zp]);
        T F = fma_t(Ct, sW[i], sw);
        F = F + (site_field ? sB[i] : b_uniform);
        const T p = fma_t(kick, F, sM[i]);
        sM[i] = p;
        if (!last) sP[i] = fma_t(drift, p, sP[i]);
      }
      __syncthreads();
    }
    // final kinetic energy and the action terms of the proposal
    {
      const int which[5] = {T_K1, T_S, T_PSI, T_PSIH, T_UT};
      unit_sums([&](int i, int x, int y, int z, double* v) {
        const double pd = (double)sM[i];
        v[0] = 0.5 * pd * pd;
        action_terms(i, x, y, z, v + 1);
      }, which, 5, acc, bad);
    }
    u128 sum[NTERM];
    const uint32_t b = block_total(acc, bad, sum);
    if (tid == 0) sFlags = finalize_trajectory(cd, st, cur, sum, b);
    __syncthreads();
    if (sFlags & REC_ACCEPT)
      for (int i = tid; i < N; i += RES_THREADS) sA[i] = sP[i];
    __syncthreads();
  }
  // the accepted field back to its buffer (finalize kept st->cur = cur)
  for (int i = tid; i < N; i += RES_THREADS) gpsi[(i % L0) + (int64_t)pitch * (i / L0)] = sA[i];
}

hipError_t launch_lattice_resident(int precision, int ndim, const ChainDev* chains, const Tile* tiles, int n_chains,
                                   int n_traj, int per_cu, hipStream_t s) {
  if (n_chains <= 0) return hipSuccess;
  if (per_cu != 1 && per_cu != 2) return hipErrorInvalidValue;
  const size_t pad = per_cu == 1 ? RES_SOLO_LDS_PAD : 0;
  if (precision == 4) {
    if (ndim == 2) lattice_resident<float, 2><<<n_chains, RES_THREADS, pad, s>>>(chains, tiles, n_traj);
    else lattice_resident<float, 3><<<n_chains, RES_THREADS, pad, s>>>(chains, tiles, n_traj);
  } else {
    if (ndim == 2) lattice_resident<double, 2><<<n_chains, RES_THREADS, pad, s>>>(chains, tiles, n_traj);
    else lattice_resident<double, 3><<<n_chains, RES_THREADS, pad, s>>>(chains, tiles, n_traj);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ launch ---

// Threads that give every SIMD of the MI355X eight waves: 256 CUs x 4 SIMDs x
// 8 waves x 64 lanes.
constexpr int64_t kFillThreads = 256 * 4 * 8 * 64;

template <typename T, int BX, int BY>
static hipError_t launch_mode2v(int mode, const ChainDev* chains, const Tile* tiles, int n_tiles, int j, int k,
                                hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  dim3 grid(n_tiles), block(BX / 4 * BY);
  switch (mode) {
    case PASS_FIRST:
      lattice_pass2v<T, BX, BY, PASS_FIRST><<<grid, block, 0, s>>>(chains, tiles, n_tiles, j, k);
      break;
    case PASS_MIDDLE:
      lattice_pass2v<T, BX, BY, PASS_MIDDLE><<<grid, block, 0, s>>>(chains, tiles, n_tiles, j, k);
      break;
    case PASS_LAST:
      lattice_pass2v<T, BX, BY, PASS_LAST><<<grid, block, 0, s>>>(chains, tiles, n_tiles, j, k);
      break;
    case PASS_MEASURE:
      lattice_pass2v<T, BX, BY, PASS_MEASURE><<<grid, block, 0, s>>>(chains, tiles, n_tiles, j, k);
      break;
    case PASS_FORCE:
      lattice_pass2v<T, BX, BY, PASS_FORCE><<<grid, block, 0, s>>>(chains, tiles, n_tiles, j, k);
      break;
    case PASS_PAIR:
      // a launch too small to give every SIMD eight waves with one thread per
      // tile quad takes two threads per quad (the ring on its own threads);
      // a large one keeps one, which leaves each thread more work in flight
      if ((int64_t)n_tiles * block.x < kFillThreads)
        lattice_pass2v_pair<T, BX, BY, 2><<<grid, dim3(2 * block.x), 0, s>>>(chains, tiles, n_tiles, j, k);
      else
        lattice_pass2v_pair<T, BX, BY, 1><<<grid, block, 0, s>>>(chains, tiles, n_tiles, j, k);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int BX, int BY, int ZR>
static hipError_t launch_mode3t(int mode, const ChainDev* chains, const Tile* tiles, int n_tiles, int j, int k,
                                hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  dim3 grid(n_tiles), block(64 * ZR);
  switch (mode) {
    case PASS_FIRST:
      lattice_pass3t<T, BX, BY, ZR, PASS_FIRST><<<grid, block, 0, s>>>(chains, tiles, n_tiles, j, k);
      break;
    case PASS_MIDDLE:
      lattice_pass3t<T, BX, BY, ZR, PASS_MIDDLE><<<grid, block, 0, s>>>(chains, tiles, n_tiles, j, k);
      break;
    case PASS_LAST:
      lattice_pass3t<T, BX, BY, ZR, PASS_LAST><<<grid, block, 0, s>>>(chains, tiles, n_tiles, j, k);
      break;
    case PASS_MEASURE:
      lattice_pass3t<T, BX, BY, ZR, PASS_MEASURE><<<grid, block, 0, s>>>(chains, tiles, n_tiles, j, k);
      break;
    case PASS_FORCE:
      lattice_pass3t<T, BX, BY, ZR, PASS_FORCE><<<grid, block, 0, s>>>(chains, tiles, n_tiles, j, k);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// 2D tiles: 64 x 16 (256 threads) for rows of 48 sites or more, 32 x 32 (256
// threads) where that wastes less of the last tile of a row, 16 x 16 (64
// threads) for small lattices.  3D boxes: 32 x 8 (or 16 x 16 by the same rule)
// in the plane, 4 planes deep, or 8 where that adds no padding planes (256
// threads per 4-plane slab).
// Tile classes: the narrower tile wherever it leaves fewer idle threads in the
// last tile of a row (row lengths just above a multiple of the wide tile); in
// 3D the 8-plane boxes (fewer halo planes per site) where L2 is a multiple of 8
// and rows are whole vector chunks (L0 a multiple of 4).
int tile_class(int ndim, int L0, int L2) {
  if (ndim == 2) {
    if (L0 < 48) return 1;
    const int r = L0 % 64;
    return (r >= 1 && r <= 32) ? 2 : 0;
  }
  const int r = L0 % 32;
  const int narrow = (r >= 1 && r <= 16) ? 1 : 0;
  const bool deep = (L2 % 8 == 0) && (L0 % 4 == 0);
  return narrow + (deep ? 2 : 0);
}

int tile_class_count(int ndim) { return ndim == 2 ? 3 : 4; }

TileShape tile_shape(int precision, int ndim, int cls) {
  (void)precision;
  if (ndim == 2) {
    if (cls == 1) return TileShape{16, 16, 1};
    if (cls == 2) return TileShape{32, 32, 1};
    return TileShape{64, 16, 1};
  }
  const int bz = cls >= 2 ? 8 : 4;
  return (cls & 1) ? TileShape{16, 16, bz} : TileShape{32, 8, bz};
}

hipError_t launch_lattice_pass(int precision, int ndim, int cls, int mode, const ChainDev* chains,
                               const Tile* tiles, int n_tiles, int j, int k, hipStream_t s) {
  if (cls == RESIDENT_CLASS || cls == RESIDENT_PHI_CLASS) {  // whole trajectories only; set-up is n_traj = 0
    if (mode != PASS_MEASURE) return hipErrorInvalidValue;
    if (cls == RESIDENT_PHI_CLASS) return launch_lattice_resident_phi(ndim, chains, tiles, n_tiles, 0, s);
    return launch_lattice_resident(precision, ndim, chains, tiles, n_tiles, 0, 2, s);
  }
  if (precision == 4) {
    if (ndim == 2) {
      if (cls == 1) return launch_mode2v<float, 16, 16>(mode, chains, tiles, n_tiles, j, k, s);
      if (cls == 2) return launch_mode2v<float, 32, 32>(mode, chains, tiles, n_tiles, j, k, s);
      return launch_mode2v<float, 64, 16>(mode, chains, tiles, n_tiles, j, k, s);
    }
    switch (cls) {
      case 1: return launch_mode3t<float, 16, 16, 4>(mode, chains, tiles, n_tiles, j, k, s);
      case 2: return launch_mode3t<float, 32, 8, 8>(mode, chains, tiles, n_tiles, j, k, s);
      case 3: return launch_mode3t<float, 16, 16, 8>(mode, chains, tiles, n_tiles, j, k, s);
      default: return launch_mode3t<float, 32, 8, 4>(mode, chains, tiles, n_tiles, j, k, s);
    }
  }
  if (ndim == 2) {
    if (cls == 1) return launch_mode2v<double, 16, 16>(mode, chains, tiles, n_tiles, j, k, s);
    if (cls == 2) return launch_mode2v<double, 32, 32>(mode, chains, tiles, n_tiles, j, k, s);
    return launch_mode2v<double, 64, 16>(mode, chains, tiles, n_tiles, j, k, s);
  }
  switch (cls) {
    case 1: return launch_mode3t<double, 16, 16, 4>(mode, chains, tiles, n_tiles, j, k, s);
    case 2: return launch_mode3t<double, 32, 8, 8>(mode, chains, tiles, n_tiles, j, k, s);
    case 3: return launch_mode3t<double, 16, 16, 8>(mode, chains, tiles, n_tiles, j, k, s);
    default: return launch_mode3t<double, 32, 8, 4>(mode, chains, tiles, n_tiles, j, k, s);
  }
}

}  // namespace ihmc
