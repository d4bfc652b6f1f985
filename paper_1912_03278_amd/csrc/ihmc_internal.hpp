// Internal data layout of the HMC runtime (device-visible structures).
#pragma once

#include <stdint.h>

namespace ihmc {

enum : uint32_t { TAG_INIT = 1u, TAG_MOM = 2u, TAG_ACC = 3u, TAG_FLIP = 4u };

enum Integrator : int32_t { LEAPFROG = 0, OMELYAN = 1 };

// Field of the chain: psi of the substituted action (eq. phi_psi_substitution,
// the hot path), phi of the inverse formulation (eq. cosh_in_exponent, whose
// force needs a linear solve per evaluation; the A/B baseline), or psi of the
// substitution phi = sqrt(J') Kt psi in eq. did_HS_trafo (h' inside the log
// cosh, no linear term; the same passes with hw != 0 and b0 = 0).
enum Form : int32_t { FORM_PSI = 0, FORM_PHI = 1, FORM_SHIFTED = 2 };

// Omelyan-Mryglod-Folk second-order minimum-norm parameter.
constexpr double kOmelyanLambda = 0.1931833275037836;

// Accumulated FP64 terms (exact fixed point, see device_common.hpp).
enum Term : int {
  T_K0 = 0,    // 1/2 p^2 of the fresh momenta (H_old)
  T_K1 = 1,    // 1/2 p^2 at the end of the trajectory (H_new)
  T_S = 2,     // action density S(psi) of the proposal
  T_PSI = 3,   // psi
  T_PSIH = 4,  // psi h'
  T_UT = 5,    // u tanh(sqrt(J') u), u = Kt psi
  NTERM = 6
};
constexpr int NPART = NTERM + 1;  // entries per tile of the partial-sum table (terms + flag words)
// Tiles per group of the two-level close: 64, or 32 for chains of more than
// 256 tiles (smaller groups complete, and are summed, while the chain's other
// blocks still run; a chain of at most 64 tiles closes in one level).
inline __host__ __device__ int part_group(uint32_t n_tiles) { return n_tiles > 256u ? 32 : 64; }
inline __host__ __device__ uint64_t part_groups(uint32_t n_tiles) {
  return (n_tiles + (uint64_t)part_group(n_tiles) - 1) / (uint64_t)part_group(n_tiles);
}

// Record written after every trajectory (64 bytes).
struct TrajRecord {
  double dH, H_old, H_new, m, abs_m, m2c, beta_eps;
  uint32_t flags;  // bit 0 accepted, bit 1 flipped, bit 2 non-finite
  uint32_t pad;
};
enum : uint32_t { REC_ACCEPT = 1u, REC_FLIP = 2u, REC_NONFINITE = 4u };

// Mutable per-chain state, updated on the device by the finalising block.
struct ChainState {
  uint64_t S_lo, S_hi;            // S(psi_cur), fixed point
  double sum_psi, sum_psih, sum_ut;  // estimator sums of psi_cur
  int32_t cur;    // buffer (0..2) holding the accepted field
  int32_t sign;   // +1, or -1 after an accepted global sign flip
  int32_t traj;   // next trajectory index
  uint32_t done;  // finished tile groups of the closing pass
  uint32_t bad;   // unused (kept for layout stability of the record fields)
  int32_t cur_bad;  // the accepted field itself has such a term (e.g. a NaN start)
  int64_t n_acc, n_nonfinite;
  double sum_exp_mdh;
  double sum_t2;  // phi form: sum of tanh^2(h' + phi) of phi_cur
  int64_t n_cg;   // phi form: CG iterations so far
};

// Immutable per-chain parameters (FP64 constants; kernels round what they need).
struct ChainDev {
  int32_t ndim, L0, L1, L2;
  int64_t N;             // lattice sites
  int32_t pitch;         // row pitch of the stored fields (L0 rounded up to 4)
  int32_t tile_cls;      // tile class of the chain's launch group (host-side choice)
  int64_t NP;            // stored elements per field: pitch * L1 * L2
  int32_t n_pass;      // force evaluations per trajectory
  int32_t integrator;
  int32_t flip_every;
  int32_t h_kind;      // 0: h = 0, 1: uniform, 2: per site
  uint32_t chain_id, n_tiles, seed_lo, seed_hi;
  double C, sqJ, Jp, b0, hp0, eps;
  double c_m, c_e, c_v;  // 1^T Kt^-1 h', h'^T Kt^-1 h', 1^T Kt^-1 1
  double hw;             // h' inside the log cosh: the uniform field of a shifted-form chain, else 0
  int32_t cap;           // capacity of the record series
  int32_t precision;     // 4 or 8 (bytes of the state type)
  int32_t p_given;       // first pass reads p instead of drawing it (diagnostic)
  int32_t write_p_last;  // last pass stores the final momenta (diagnostic)
  int32_t n_therm;       // trajectories before this index stay out of the summary counters
  int32_t form;          // FORM_PSI or FORM_PHI
  void* psi;             // rotating field buffers of NP values: LAT_BUFFERS (lattice) or 3 (dense)
  void* p;               // NP state values
  const void* b;         // NP state values h'/sqrt(J') (per-site field) or null
  const double* hp;      // NP FP64 h' (per-site field) or null
  TrajRecord* rec;       // cap records
  const uint8_t* replay; // forced decisions (test hook) or null
  ChainState* st;
  uint64_t* part;   // n_tiles x NPART fixed-point entries (block sums of the current trajectory)
  uint64_t* gsum;   // part_groups(n_tiles) x NPART group sums
  uint32_t* gcnt;   // part_groups(n_tiles) tile counters, zero between passes
};

// Bytes of a chain's partial-sum table, group sums and group counters.
inline __host__ __device__ uint64_t partials_bytes(uint32_t n_tiles) {
  const uint64_t ng = part_groups(n_tiles);
  return ((uint64_t)n_tiles * NPART * 16 + 255) / 256 * 256 + (ng * NPART * 16 + 255) / 256 * 256 +
         (ng * 4 + 255) / 256 * 256;
}

// Stored index of logical site i = x + L0 (y + L1 z).
inline __host__ __device__ int64_t stored_index(const ChainDev& cd, int64_t i) {
  const int64_t x = i % cd.L0, r = i / cd.L0;
  return x + (int64_t)cd.pitch * r;
}

// One work tile of a lattice pass.
struct Tile {
  int32_t chain;
  int32_t x0, y0, z0;
};

// Kick and drift coefficients of pass j (0 <= j < n_pass).
inline __host__ __device__ void pass_coeffs(const ChainDev& cd, int j, double& kick, double& drift) {
  const double e = cd.eps;
  const int last = cd.n_pass - 1;
  if (cd.integrator == OMELYAN) {
    const double l = kOmelyanLambda;
    if (j == 0 || j == last) kick = l * e;
    else if (j & 1) kick = (1.0 - 2.0 * l) * e;
    else kick = 2.0 * l * e;
    drift = (j == last) ? 0.0 : 0.5 * e;
  } else {
    kick = (j == 0 || j == last) ? 0.5 * e : e;
    drift = (j == last) ? 0.0 : e;
  }
}

// Field buffers of a lattice chain (four): the accepted field sits in buffer
// `cur`; launch k of a trajectory (k = 0 the first pass; a launch may fuse two
// leap-frog steps) reads lat_in_buf and writes lat_out_buf, cycling through the
// three other buffers, so no launch writes the buffer it reads.
constexpr int LAT_BUFFERS = 4;
inline __host__ __device__ int lat_in_buf(int cur, int k) { return k == 0 ? cur : (cur + 1 + (k - 1) % 3) % 4; }
inline __host__ __device__ int lat_out_buf(int cur, int k) { return (cur + 1 + k % 3) % 4; }

// Momentum buffers of a lattice chain (two).  In 2D, launch k >= 1 reads
// buffer lat_p_in(k) and writes lat_p_out(k): a launch that fuses two steps
// reads the momenta of neighbouring tiles, so it must not write the buffer it
// reads.  The first pass, the last pass and the force pass use buffer 0 (where
// given momenta are read and final ones exported); 3D passes update buffer 0
// in place.
constexpr int LAT_P_BUFFERS = 2;
inline __host__ __device__ int lat_p_in(int k) { return k == 0 ? 0 : (k - 1) & 1; }
inline __host__ __device__ int lat_p_out(int k) { return k & 1; }

// Dense chains (three buffers): buffer read by pass j when the accepted field
// sits in buffer `cur`.
inline __host__ __device__ int pass_in_buf(int cur, int j) {
  if (j == 0) return cur;
  return (j & 1) ? (cur + 1) % 3 : (cur + 2) % 3;
}
inline __host__ __device__ int pass_out_buf(int cur, int j) {
  return (j & 1) ? (cur + 2) % 3 : (cur + 1) % 3;
}

}  // namespace ihmc
