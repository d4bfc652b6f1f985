// Host runtime and C ABI (include/ihmc.h): context, device arena, chain set-up
// (Sec. 2 constants and the initial field), the per-trajectory launch sequence
// captured into a HIP graph, and result export.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ihmc.h"
#include "device_common.hpp"
#include "lattice_kernels.hpp"
#include "runtime_internal.hpp"

namespace ihmc {

// ------------------------------------------------------------------ errors ---

static thread_local std::string g_err;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(ihmc_ctx* ctx, hipError_t e, const char* where) {
  if (ctx) ctx->dead = true;
  return set_error(IHMC_E_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

// ------------------------------------------------------------------- arena ---

void* Arena::alloc(uint64_t bytes) {
  bytes = (bytes + 255ull) & ~255ull;
  if (bytes == 0) bytes = 256;
  std::lock_guard<std::mutex> lk(mu);
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= bytes) {
      const uint64_t off = it->first, rem = it->second - bytes;
      free_.erase(it);
      if (rem) free_[off + bytes] = rem;
      live_[off] = bytes;
      used += bytes;
      return base + off;
    }
  }
  return nullptr;
}

void Arena::release(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(mu);
  const uint64_t off = (uint64_t)((char*)p - base);
  auto it = live_.find(off);
  if (it == live_.end()) return;
  uint64_t sz = it->second;
  live_.erase(it);
  used -= sz;
  uint64_t start = off;
  auto nx = free_.lower_bound(off);
  if (nx != free_.end() && nx->first == off + sz) {
    sz += nx->second;
    free_.erase(nx);
  }
  auto pv = free_.lower_bound(off);
  if (pv != free_.begin()) {
    --pv;
    if (pv->first + pv->second == off) {
      start = pv->first;
      sz += pv->second;
      free_.erase(pv);
    }
  }
  free_[start] = sz;
}

// ---------------------------------------------------------- set-up kernels ---

// h' = beta h (FP64) and h'/sqrt(J') (state precision) at the stored indices.
template <typename T>
__global__ void k_field_setup(const ChainDev* cds, int ci, const double* h, double beta) {
  const ChainDev& cd = cds[ci];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= cd.N) return;
  const int64_t k = stored_index(cd, i);
  const double hp = beta * h[i];
  ((double*)cd.hp)[k] = hp;
  ((T*)cd.b)[k] = (T)(hp / cd.sqJ);
}

// Starting field: psi0 (logical layout) or the TAG_INIT normals, plus `shift`
// (logical layout, or null) before the rounding to the state type.
template <typename T>
__global__ void k_init_psi(const ChainDev* cds, int ci, const double* psi0, const double* shift) {
  const ChainDev& cd = cds[ci];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= cd.N) return;
  T* psi = (T*)cd.psi;
  double v = psi0 ? psi0[i] : normal_at(cd, 0u, TAG_INIT, i);
  if (shift) v += shift[i];
  psi[stored_index(cd, i)] = (T)v;
}

// x /= s over n values (the translation of a shifted-form chain from Kt^-1 h').
__global__ void k_scale(double* x, int64_t n, double s) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] /= s;
}

// Starting field of a phi-form chain without a given one: the substitution
// phi0 = sqrt(J') Kt psi0 - h' (Sec. 2) of the TAG_INIT normals psi0 that a
// psi-form chain of the same seed starts from (FP64 state).
__global__ void k_init_phi(const ChainDev* cds, int ci) {
  const ChainDev& cd = cds[ci];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= cd.N) return;
  const int L0 = cd.L0, L1 = cd.L1, L2 = cd.L2;
  const int x = (int)(i % L0), y = (int)((i / L0) % L1), z = (int)(i / ((int64_t)L0 * L1));
  auto at = [&](int a, int b, int c) { return normal_at(cd, 0u, TAG_INIT, a + (int64_t)L0 * (b + (int64_t)L1 * c)); };
  double u = cd.C * at(x, y, z);
  u += at((x + 1) % L0, y, z);
  u += at((x + L0 - 1) % L0, y, z);
  u += at(x, (y + 1) % L1, z);
  u += at(x, (y + L1 - 1) % L1, z);
  if (cd.ndim == 3) {
    u += at(x, y, (z + 1) % L2);
    u += at(x, y, (z + L2 - 1) % L2);
  }
  const int64_t k = stored_index(cd, i);
  const double hp = cd.h_kind == 2 ? cd.hp[k] : cd.hp0;
  ((double*)cd.psi)[k] = cd.sqJ * u - hp;
}

// Logical <-> stored layout of one field (p or F).
template <typename T>
__global__ void k_import(const ChainDev* cds, int ci, T* dst, const double* src) {
  const ChainDev& cd = cds[ci];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < cd.N) dst[stored_index(cd, i)] = (T)src[i];
}

template <typename T>
__global__ void k_export_psi(const ChainDev* cds, int ci, double* out) {
  const ChainDev& cd = cds[ci];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= cd.N) return;
  const ChainState* st = cd.st;
  const double v = (double)((const T*)cd.psi)[(int64_t)st->cur * cd.NP + stored_index(cd, i)];
  out[i] = st->sign < 0 ? -v : v;
}

template <typename T>
__global__ void k_export(const ChainDev* cds, int ci, double* dst, const T* src) {
  const ChainDev& cd = cds[ci];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < cd.N) dst[i] = (double)src[stored_index(cd, i)];
}

__global__ void k_zero_state(ChainState* st) {
  uint64_t* w = (uint64_t*)st;
  const int nw = (int)(sizeof(ChainState) / 8);
  for (int i = threadIdx.x; i < nw; i += blockDim.x) w[i] = 0ull;
  __syncthreads();
  if (threadIdx.x == 0) st->sign = 1;
}

__global__ void k_philox_words(int64_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint4 c = make_uint4(ctr[4 * k], ctr[4 * k + 1], ctr[4 * k + 2], ctr[4 * k + 3]);
  const uint4 r = philox4x32_10(c, key[2 * k], key[2 * k + 1]);
  out[4 * k] = r.x;
  out[4 * k + 1] = r.y;
  out[4 * k + 2] = r.z;
  out[4 * k + 3] = r.w;
}

// Normals of sites 0..n-1 exactly as a pass of state type T draws them (one
// pair per thread).
template <typename T>
__global__ void k_philox_normals(ChainDev cd, uint32_t traj, uint32_t tag, int64_t n, double* out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (2 * i >= n) return;
  T z0, z1;
  normal_pair<T>(cd, traj, tag, i, z0, z1);
  out[2 * i] = (double)z0;
  if (2 * i + 1 < n) out[2 * i + 1] = (double)z1;
}

// Deterministic block-wide FP64 sum (fixed order), result broadcast to all threads.
__device__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) t += sh[w];
  return t;
}

__device__ void lattice_apply_global(const ChainDev& cd, const double* x, double* y) {
  const int L0 = cd.L0, L1 = cd.L1, L2 = cd.L2;
  for (int64_t s = threadIdx.x; s < cd.N; s += blockDim.x) {
    const int gx = (int)(s % L0);
    const int gy = (int)((s / L0) % L1);
    const int gz = (int)(s / ((int64_t)L0 * L1));
    auto at = [&](int a, int b, int c) { return x[a + (int64_t)L0 * (b + (int64_t)L1 * c)]; };
    double acc = (at((gx + L0 - 1) % L0, gy, gz) + at((gx + 1) % L0, gy, gz)) +
                 (at(gx, (gy + L1 - 1) % L1, gz) + at(gx, (gy + 1) % L1, gz));
    if (cd.ndim == 3) acc += at(gx, gy, (gz + L2 - 1) % L2) + at(gx, gy, (gz + 1) % L2);
    y[s] = cd.C * x[s] + acc;
  }
}

// Per-site field: h'^T Kt^-1 h' by conjugate gradients (Sec. 2: solve Kt x = h'
// instead of inverting) and 1^T Kt^-1 h' = sum h' / (n0 + C).  One block per chain.
__global__ __launch_bounds__(256) void k_field_cg(ChainDev* cds, const int* which, double* work,
                                                  const int64_t* woff) {
  __shared__ double sh[8];
  ChainDev& cd = cds[which[blockIdx.x]];
  const int64_t N = cd.N;
  double* x = work + woff[blockIdx.x];
  double* r = x + N;
  double* d = r + N;
  double* q = d + N;
  const double* hp = cd.hp;  // stored layout; the CG vectors use the logical one
  double hs = 0.0, rr = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
    const double v = hp[stored_index(cd, i)];
    x[i] = 0.0;
    r[i] = v;
    d[i] = v;
    hs += v;
    rr += v * v;
  }
  hs = block_sum(hs, sh);
  rr = block_sum(rr, sh);
  const double stop = 1e-30 * rr;
  for (int it = 0; it < 20000 && rr > stop; ++it) {
    __syncthreads();
    lattice_apply_global(cd, d, q);
    __syncthreads();
    double dq = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) dq += d[i] * q[i];
    dq = block_sum(dq, sh);
    const double alpha = rr / dq;
    double rn = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
      x[i] += alpha * d[i];
      r[i] -= alpha * q[i];
      rn += r[i] * r[i];
    }
    rn = block_sum(rn, sh);
    const double beta = rn / rr;
    rr = rn;
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) d[i] = r[i] + beta * d[i];
  }
  __syncthreads();
  double ce = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) ce += hp[stored_index(cd, i)] * x[i];
  ce = block_sum(ce, sh);
  if (threadIdx.x == 0) {
    cd.c_e = ce;
    cd.c_m = hs / (2.0 * cd.ndim + cd.C);
  }
}

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Descriptor of one lattice chain (no device memory yet).
void describe_chain(const ihmc_lattice& l, const ihmc_run& r, int flags, int cls, ChainDev& c) {
  std::memset(&c, 0, sizeof c);
  c.ndim = l.ndim;
  c.L0 = l.L[0];
  c.L1 = l.L[1];
  c.L2 = l.ndim == 3 ? l.L[2] : 1;
  c.N = lattice_sites(l);
  c.pitch = (c.L0 + 3) & ~3;
  c.NP = (int64_t)c.pitch * c.L1 * c.L2;
  c.integrator = r.integrator;
  c.n_pass = r.integrator == OMELYAN ? 2 * r.n_md + 1 : r.n_md + 1;
  c.flip_every = r.flip_every;
  c.h_kind = l.h_len == 0 ? 0 : (l.h_len == 1 ? 1 : 2);
  c.chain_id = (uint32_t)r.chain_id;
  c.seed_lo = (uint32_t)r.seed;
  c.seed_hi = (uint32_t)(r.seed >> 32);
  c.Jp = l.beta * l.J;
  c.sqJ = std::sqrt(c.Jp);
  c.C = l.C;
  c.eps = r.traj_len / r.n_md;
  c.hp0 = c.h_kind == 1 ? l.beta * l.h[0] : 0.0;
  c.b0 = c.h_kind == 1 ? c.hp0 / c.sqJ : 0.0;
  const double n0c = 2.0 * l.ndim + l.C;
  // Kt 1 = (n0 + C) 1 on the periodic lattice (eq. hKh_for_constant_h)
  c.c_v = (double)c.N / n0c;
  c.c_m = c.h_kind == 1 ? (double)c.N * c.hp0 / n0c : 0.0;
  c.c_e = c.h_kind == 1 ? (double)c.N * c.hp0 * c.hp0 / n0c : 0.0;
  c.cap = r.n_traj;
  c.precision = r.precision;
  c.p_given = (flags & BUILD_P_GIVEN) ? 1 : 0;
  c.write_p_last = (flags & BUILD_WRITE_P) ? 1 : 0;
  c.n_therm = r.n_therm;
  c.form = r.form;
  c.hw = 0.0;
  if (r.form == FORM_SHIFTED && c.h_kind == 2) {
    // a per-site field: the chain runs as a paper-form chain in coordinates
    // translated by Kt^-1 h'/sqrt(J') (set up by Chains::build)
    c.form = FORM_PSI;
  } else if (r.form == FORM_SHIFTED) {
    // h' moves inside the log cosh; the linear term and the Kt^-1 constants of
    // the estimators drop (h' itself stays for the psi.h' estimator sum)
    c.hw = c.hp0;
    c.b0 = 0.0;
    c.c_m = 0.0;
    c.c_e = 0.0;
  }
  c.tile_cls = cls;
  c.n_tiles = chain_tile_count(c);
}

int choose_class(ihmc_ctx* ctx, const ihmc_lattice& l, int precision, int flags, int form) {
  if (form == FORM_PHI) return RESIDENT_PHI_CLASS;
  const int64_t N = lattice_sites(l);
  const bool site_field = !(l.h_len == 0 || l.h_len == 1);
  const int64_t fit = resident_max_sites(precision, site_field);
  const int64_t lim = ctx->resident_sites < 0 ? fit : std::min(fit, ctx->resident_sites);
  (void)flags;
  if (flags == 0 && N <= lim) return RESIDENT_CLASS;
  return ctx->tune.class_for(tile_key(l, precision));
}

// Tiles of one chain in the tile shape of its launch group (one per resident chain).
uint32_t chain_tile_count(const ChainDev& c) {
  if (c.tile_cls < 0) return 1u;  // LDS-resident: one workgroup per chain
  const TileShape ts = tile_shape(c.precision, c.ndim, c.tile_cls);
  const uint32_t nz = c.ndim == 3 ? (uint32_t)((c.L2 + ts.bz - 1) / ts.bz) : 1u;
  return nz * (uint32_t)((c.L1 + ts.by - 1) / ts.by) * (uint32_t)((c.L0 + ts.bx - 1) / ts.bx);
}

// Launch groups of equal (precision, ndim, tile class) over the chains
// `members` (indices into cd), each sorted by pass count (descending), and
// their tiles appended to `tiles` (group tile offsets relative to its start).
void plan_groups(const std::vector<ChainDev>& cd, const std::vector<int>& members, std::vector<Group>& groups,
                 std::vector<Tile>& tiles, bool fuse_steps) {
  const int base = (int)tiles.size();
  std::map<std::tuple<int, int, int>, std::vector<int>> byk;
  for (int i : members)
    byk[std::make_tuple(cd[i].precision, cd[i].ndim, cd[i].tile_cls)].push_back(i);
  for (auto& kv : byk) {
    Group g;
    g.prec = std::get<0>(kv.first);
    g.ndim = std::get<1>(kv.first);
    g.cls = std::get<2>(kv.first);
    g.order = kv.second;
    std::stable_sort(g.order.begin(), g.order.end(), [&](int a, int b) { return cd[a].n_pass > cd[b].n_pass; });
    const bool resident = (g.cls < 0);
    g.pair = fuse_steps && g.ndim == 2 && !resident;
    const TileShape ts = resident ? TileShape{1, 1, 1} : tile_shape(g.prec, g.ndim, g.cls);
    g.tile_off = (int)tiles.size() - base;
    for (int ci : g.order) {
      const ChainDev& c = cd[ci];
      g.tile_begin.push_back((int)tiles.size() - base - g.tile_off);
      if (resident) {
        tiles.push_back(Tile{ci, 0, 0, 0});
      } else {
        for (int z = 0; z < c.L2; z += (g.ndim == 3 ? ts.bz : 1))
          for (int y = 0; y < c.L1; y += ts.by)
            for (int x = 0; x < c.L0; x += ts.bx) tiles.push_back(Tile{ci, x, y, z});
      }
      g.n_pass.push_back(c.n_pass);
    }
    g.tile_begin.push_back((int)tiles.size() - base - g.tile_off);
    g.max_pass = cd[g.order[0]].n_pass;
    groups.push_back(g);
  }
}

// Events one round of the plan needs: the fork, and one join per group.
size_t round_events(const std::vector<Group>& groups) { return 1 + groups.size(); }

// ------------------------------------------------------------ validation ---

int64_t lattice_sites(const ihmc_lattice& l) {
  int64_t n = 1;
  for (int i = 0; i < l.ndim; ++i) n *= l.L[i];
  return n;
}

int validate(const ihmc_lattice& l, const ihmc_run& r, int idx) {
  if (l.ndim == 1) return set_error(IHMC_E_UNSUPPORTED, "chain %d: 1D lattices are not supported on the GPU", idx);
  if (l.ndim != 2 && l.ndim != 3) return set_error(IHMC_E_INVAL, "chain %d: ndim must be 2 or 3", idx);
  for (int i = 0; i < l.ndim; ++i)
    if (l.L[i] < 3 || l.L[i] > (1 << 20)) return set_error(IHMC_E_INVAL, "chain %d: L[%d] must be in [3, 2^20]", idx, i);
  if (!(l.beta * l.J > 0.0) || !std::isfinite(l.beta * l.J))
    return set_error(IHMC_E_INVAL, "chain %d: J' = beta*J must be positive and finite", idx);
  if (!(l.C > 2.0 * l.ndim) || !std::isfinite(l.C))
    return set_error(IHMC_E_INVAL, "chain %d: C must exceed 2*ndim so that J' Kt is positive definite", idx);
  const int64_t N = lattice_sites(l);
  if (N >= (int64_t(1) << 33)) return set_error(IHMC_E_INVAL, "chain %d: too many sites", idx);
  if (!(l.h_len == 0 || l.h_len == 1 || l.h_len == N))
    return set_error(IHMC_E_INVAL, "chain %d: h_len must be 0, 1 or N", idx);
  if (l.h_len > 0 && !l.h) return set_error(IHMC_E_INVAL, "chain %d: h is NULL", idx);
  if (r.n_md < 1) return set_error(IHMC_E_INVAL, "chain %d: n_md must be >= 1", idx);
  if (r.n_traj < 0) return set_error(IHMC_E_INVAL, "chain %d: n_traj must be >= 0", idx);
  if (!(r.traj_len > 0.0) || !std::isfinite(r.traj_len))
    return set_error(IHMC_E_INVAL, "chain %d: traj_len must be positive", idx);
  if (r.integrator != LEAPFROG && r.integrator != OMELYAN)
    return set_error(IHMC_E_INVAL, "chain %d: unknown integrator", idx);
  if (r.precision != 4 && r.precision != 8) return set_error(IHMC_E_INVAL, "chain %d: precision must be 4 or 8", idx);
  if (r.flip_every < 0) return set_error(IHMC_E_INVAL, "chain %d: flip_every must be >= 0", idx);
  if (r.n_therm < 0) return set_error(IHMC_E_INVAL, "chain %d: n_therm must be >= 0", idx);
  if (r.form != FORM_PSI && r.form != FORM_PHI && r.form != FORM_SHIFTED)
    return set_error(IHMC_E_INVAL, "chain %d: unknown form", idx);
  if (r.form == FORM_SHIFTED && r.flip_every > 0) {
    bool field = false;
    for (int64_t k = 0; k < l.h_len && !field; ++k) field = l.h[k] != 0.0;
    if (field) return set_error(IHMC_E_INVAL, "chain %d: psi -> -psi is no symmetry of the shifted form at h != 0", idx);
  }
  if (r.form == FORM_PHI) {
    if (r.precision != 8 || r.integrator != LEAPFROG || r.flip_every != 0)
      return set_error(IHMC_E_UNSUPPORTED, "chain %d: the phi form runs FP64 leap-frog chains without flips", idx);
    const bool site_field = !(l.h_len == 0 || l.h_len == 1);
    if (N > resident_phi_max_sites(site_field))
      return set_error(IHMC_E_UNSUPPORTED, "chain %d: the phi form takes chains of at most %d sites", idx,
                       resident_phi_max_sites(site_field));
  }
  return IHMC_OK;
}

}  // namespace ihmc

using namespace ihmc;

// =========================================================== C ABI: context ===

extern "C" const char* ihmc_last_error(void) { return g_err.c_str(); }

extern "C" int ihmc_ctx_create(int32_t device, uint64_t arena_bytes, ihmc_alloc_fn alloc, ihmc_free_fn free_fn,
                               void* user, ihmc_ctx** out) {
  if (!out) return set_error(IHMC_E_INVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return set_error(IHMC_E_DEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return set_error(IHMC_E_INVAL, "device %d out of range", device);
  if ((alloc == nullptr) != (free_fn == nullptr)) return set_error(IHMC_E_INVAL, "alloc and free must both be set");
  if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
  if (arena_bytes == 0) arena_bytes = 1ull << 30;
  arena_bytes = (arena_bytes + 255ull) & ~255ull;
  ihmc_ctx* c = new (std::nothrow) ihmc_ctx();
  if (!c) return set_error(IHMC_E_NOMEM, "host allocation failed");
  c->device = device;
  c->af = alloc;
  c->ff = free_fn;
  c->user = user;
  void* base = nullptr;
  if (alloc) {
    base = alloc(arena_bytes, user);
    if (!base) {
      delete c;
      return set_error(IHMC_E_NOMEM, "allocator callback failed for %llu bytes", (unsigned long long)arena_bytes);
    }
  } else if ((e = hipMalloc(&base, arena_bytes)) != hipSuccess) {
    delete c;
    return set_error(IHMC_E_NOMEM, "hipMalloc(%llu): %s", (unsigned long long)arena_bytes, hipGetErrorString(e));
  }
  c->arena.base = (char*)base;
  c->arena.size = arena_bytes;
  c->arena.free_[0] = arena_bytes;
  if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess) {
    if (alloc) free_fn(base, user);
    else hipFree(base);
    delete c;
    return hip_fail(nullptr, e, "hipStreamCreate");
  }
  // the allocation-free entry point's scratch on this device
  {
    const int rc = noalloc_scratch_init(device, &c->scratch);
    if (rc) {
      ihmc_ctx_destroy(c);
      return rc;
    }
  }
  // tile classes chosen earlier, when a cache file is named and present
  const char* cache = std::getenv("IHMC_TUNE_CACHE");
  if (cache && *cache) {
    if (FILE* f = std::fopen(cache, "r")) {
      std::fclose(f);
      const int rc = tune_load(c->tune, cache);
      if (rc) {
        ihmc_ctx_destroy(c);
        return rc;
      }
    }
  }
  *out = c;
  return IHMC_OK;
}

extern "C" void ihmc_ctx_destroy(ihmc_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  hipStreamDestroy(c->stream);
  if (c->af) c->ff(c->arena.base, c->user);
  else hipFree(c->arena.base);
  delete c;
}

extern "C" void* ihmc_ctx_stream(ihmc_ctx* c) { return c ? (void*)c->stream : nullptr; }

extern "C" int ihmc_ctx_sync(ihmc_ctx* c) {
  if (!c) return set_error(IHMC_E_INVAL, "ctx is NULL");
  hipSetDevice(c->device);
  hipError_t e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? IHMC_OK : hip_fail(c, e, "hipStreamSynchronize");
}

extern "C" int ihmc_ctx_set_resident(ihmc_ctx* c, int64_t max_sites, int64_t* fp32_fit, int64_t* fp64_fit) {
  if (!c) return set_error(IHMC_E_INVAL, "ctx is NULL");
  c->resident_sites = max_sites < 0 ? -1 : max_sites;
  if (fp32_fit) *fp32_fit = resident_max_sites(4, false);
  if (fp64_fit) *fp64_fit = resident_max_sites(8, false);
  return IHMC_OK;
}

extern "C" int ihmc_ctx_set_step_fusion(ihmc_ctx* c, int32_t on) {
  if (!c) return set_error(IHMC_E_INVAL, "ctx is NULL");
  c->fuse_steps = on ? 1 : 0;
  return IHMC_OK;
}

extern "C" int ihmc_ctx_memory(ihmc_ctx* c, uint64_t* used, uint64_t* total) {
  if (!c) return set_error(IHMC_E_INVAL, "ctx is NULL");
  if (used) *used = c->arena.used;
  if (total) *total = c->arena.size;
  return IHMC_OK;
}

// ============================================================ chain objects ===

namespace ihmc {

void* Chains::dalloc(uint64_t bytes) {
  void* p = ctx->arena.alloc(bytes);
  if (p) allocs.push_back(p);
  return p;
}

Chains::~Chains() {
  if (gexec) hipGraphExecDestroy(gexec);
  if (graph) hipGraphDestroy(graph);
  for (hipEvent_t ev : events) hipEventDestroy(ev);
  for (hipStream_t st : side) hipStreamDestroy(st);
  for (void* p : allocs) ctx->arena.release(p);
}



int Chains::build(int32_t n_, const ihmc_lattice* lats, const ihmc_run* runs, int flags) {
  n = n_;
  cd.resize(n);
  delta.assign(n, std::vector<double>());
  s_offset.assign(n, 0.0);
  base.assign(n, 0);
  hipStream_t s = ctx->stream;
  std::vector<void*> temps;
  auto tmp_alloc = [&](uint64_t bytes) {
    void* p = ctx->arena.alloc(bytes);
    if (p) temps.push_back(p);
    return p;
  };
  auto cleanup = [&]() {
    hipStreamSynchronize(s);
    for (void* p : temps) ctx->arena.release(p);
    temps.clear();
  };
  for (int i = 0; i < n; ++i) {
    const ihmc_lattice& l = lats[i];
    const ihmc_run& r = runs[i];
    int rc = validate(l, r, i);
    if (rc) return rc;
    ChainDev& c = cd[i];
    describe_chain(l, r, flags, choose_class(ctx, l, r.precision, flags, r.form), c);
    const int64_t N = c.N, NP = c.NP;
    const int64_t pb = r.precision;
    c.psi = dalloc((uint64_t)LAT_BUFFERS * NP * pb);
    c.p = dalloc((uint64_t)LAT_P_BUFFERS * NP * pb);
    c.rec = (TrajRecord*)dalloc(sizeof(TrajRecord) * (uint64_t)std::max(1, r.n_traj));
    c.st = (ChainState*)dalloc(sizeof(ChainState));
    void* pblk = dalloc(partials_bytes(c.n_tiles));
    if (pblk) HIPCHK(setup_partials(c, pblk, s), "partials");
    if (!c.psi || !c.p || !c.rec || !c.st || !pblk) {
      cleanup();
      return set_error(IHMC_E_NOMEM, "chain %d: device arena exhausted (%llu of %llu bytes in use)", i,
                       (unsigned long long)ctx->arena.used, (unsigned long long)ctx->arena.size);
    }
    if (r.replay_accept && r.n_traj > 0) {
      uint8_t* d = (uint8_t*)dalloc((uint64_t)r.n_traj);
      if (!d) {
        cleanup();
        return set_error(IHMC_E_NOMEM, "chain %d: arena exhausted", i);
      }
      HIPCHK(hipMemcpyAsync(d, r.replay_accept, (size_t)r.n_traj, hipMemcpyHostToDevice, s), "replay upload");
      c.replay = d;
    }
    if (c.h_kind == 2) {
      c.hp = (double*)dalloc(8 * NP);
      c.b = dalloc(NP * pb);
      if (!c.hp || !c.b) {
        cleanup();
        return set_error(IHMC_E_NOMEM, "chain %d: arena exhausted", i);
      }
    }
    k_zero_state<<<1, 256, 0, s>>>(c.st);
  }
  d_cd = (ChainDev*)dalloc(sizeof(ChainDev) * (uint64_t)n);
  if (!d_cd) {
    cleanup();
    return set_error(IHMC_E_NOMEM, "arena exhausted (chain table)");
  }

  // ---- groups of equal (precision, ndim, tile class), chains sorted by passes (descending)
  std::vector<Tile> all_tiles;
  {
    std::vector<int> members(n);
    for (int i = 0; i < n; ++i) members[i] = i;
    plan_groups(cd, members, groups, all_tiles, ctx->fuse_steps != 0);
  }
  // streams and events of the per-round fork/join (default priority)
  {
    const size_t n_ev = round_events(groups);
    for (size_t k = 0; k < groups.size(); ++k) {
      hipStream_t st = nullptr;
      HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "side stream");
      side.push_back(st);
    }
    for (size_t k = 0; k < n_ev; ++k) {
      hipEvent_t ev = nullptr;
      HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
      events.push_back(ev);
    }
  }
  d_tiles = (Tile*)dalloc(sizeof(Tile) * all_tiles.size());
  if (!d_tiles) {
    cleanup();
    return set_error(IHMC_E_NOMEM, "arena exhausted (tile table)");
  }
  HIPCHK(hipMemcpyAsync(d_tiles, all_tiles.data(), sizeof(Tile) * all_tiles.size(), hipMemcpyHostToDevice, s),
         "tile upload");
  HIPCHK(hipMemcpyAsync(d_cd, cd.data(), sizeof(ChainDev) * (uint64_t)n, hipMemcpyHostToDevice, s), "chain upload");

  // ---- per-site fields into the stored layout
  for (int i = 0; i < n; ++i) {
    if (cd[i].h_kind != 2) continue;
    const int64_t N = cd[i].N;
    double* t = (double*)tmp_alloc(8 * (uint64_t)N);
    if (!t) {
      cleanup();
      return set_error(IHMC_E_NOMEM, "arena exhausted (field staging)");
    }
    HIPCHK(hipMemcpyAsync(t, lats[i].h, 8 * N, hipMemcpyHostToDevice, s), "h upload");
    if (cd[i].precision == 4) k_field_setup<float><<<nblk(N), 256, 0, s>>>(d_cd, i, t, lats[i].beta);
    else k_field_setup<double><<<nblk(N), 256, 0, s>>>(d_cd, i, t, lats[i].beta);
    HIPCHK(hipGetLastError(), "k_field_setup");
  }

  // ---- per-site field constants by CG (one block per chain)
  std::vector<double*> shift(n, nullptr);
  std::vector<int> cg_idx;
  std::vector<int64_t> cg_off;
  int64_t cg_total = 0;
  for (int i = 0; i < n; ++i)
    if (cd[i].h_kind == 2) {
      cg_idx.push_back(i);
      cg_off.push_back(cg_total);
      cg_total += 4 * cd[i].N;
    }
  if (!cg_idx.empty()) {
    double* work = (double*)tmp_alloc(8 * (uint64_t)cg_total);
    int* didx = (int*)tmp_alloc(sizeof(int) * cg_idx.size());
    int64_t* doff = (int64_t*)tmp_alloc(sizeof(int64_t) * cg_off.size());
    if (!work || !didx || !doff) {
      cleanup();
      return set_error(IHMC_E_NOMEM, "arena exhausted (CG work space)");
    }
    HIPCHK(hipMemcpyAsync(didx, cg_idx.data(), sizeof(int) * cg_idx.size(), hipMemcpyHostToDevice, s), "cg idx");
    HIPCHK(hipMemcpyAsync(doff, cg_off.data(), sizeof(int64_t) * cg_off.size(), hipMemcpyHostToDevice, s), "cg off");
    k_field_cg<<<(unsigned)cg_idx.size(), 256, 0, s>>>(d_cd, didx, work, doff);
    HIPCHK(hipGetLastError(), "k_field_cg");
    // shifted-form chains with this field: delta = Kt^-1 h' / sqrt(J') (the CG's x)
    for (size_t j = 0; j < cg_idx.size(); ++j) {
      const int i = cg_idx[j];
      if (runs[i].form != FORM_SHIFTED) continue;
      shift[i] = work + cg_off[j];
      k_scale<<<nblk(cd[i].N), 256, 0, s>>>(shift[i], cd[i].N, cd[i].sqJ);
      HIPCHK(hipGetLastError(), "k_scale");
    }
  }

  // ---- initial field and its action
  for (int i = 0; i < n; ++i) {
    const ihmc_run& r = runs[i];
    const int64_t N = cd[i].N;
    const double* src = nullptr;
    if (r.psi0) {
      double* t = (double*)tmp_alloc(8 * (uint64_t)N);
      if (!t) {
        cleanup();
        return set_error(IHMC_E_NOMEM, "arena exhausted (psi0 staging)");
      }
      HIPCHK(hipMemcpyAsync(t, r.psi0, 8 * N, hipMemcpyHostToDevice, s), "psi0 upload");
      src = t;
    }
    if (cd[i].form == FORM_PHI && !src) k_init_phi<<<nblk(N), 256, 0, s>>>(d_cd, i);
    else if (cd[i].precision == 4) k_init_psi<float><<<nblk(N), 256, 0, s>>>(d_cd, i, src, shift[i]);
    else k_init_psi<double><<<nblk(N), 256, 0, s>>>(d_cd, i, src, shift[i]);
    HIPCHK(hipGetLastError(), "k_init_psi");
  }
  for (auto& g : groups) {
    HIPCHK(launch_lattice_pass(g.prec, g.ndim, g.cls, PASS_MEASURE, d_cd, d_tiles + g.tile_off, g.tile_begin.back(), 0, 0, s),
           "measure pass");
  }
  hipError_t e = hipStreamSynchronize(s);
  // translated chains: delta and the action offset h'.Kt^-1 h'/(2J') on the host
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    if (!shift[i]) continue;
    delta[i].resize((size_t)cd[i].N);
    e = hipMemcpy(delta[i].data(), shift[i], 8 * (uint64_t)cd[i].N, hipMemcpyDeviceToHost);
    double ce = 0.0;
    if (e == hipSuccess) e = hipMemcpy(&ce, &d_cd[i].c_e, sizeof ce, hipMemcpyDeviceToHost);
    s_offset[i] = ce / (2.0 * cd[i].Jp);
  }
  cleanup();
  if (e != hipSuccess) return hip_fail(ctx, e, "chain set-up");
  return IHMC_OK;
}

// One launch running n_traj whole trajectories (0: the set-up measurement) of
// every chain of an LDS-resident group; per_cu as in launch_lattice_resident.
hipError_t launch_resident_group(const Group& g, const ChainDev* d_cd, const Tile* t, int n, int n_traj,
                                 int per_cu, hipStream_t s) {
  if (g.cls == RESIDENT_PHI_CLASS) return launch_lattice_resident_phi(g.ndim, d_cd, t, n, n_traj, s);
  return launch_lattice_resident(g.prec, g.ndim, d_cd, t, n, n_traj, per_cu, s);
}

// Enqueue target of a round plan: the HIP stream operations, or (dry) a count
// of the events the plan takes, with no HIP call at all.  Every event the plan
// takes comes from the pool; a plan that would take more than the pool holds
// fails with hipErrorInvalidValue before it records anything past the end.
struct RoundSink {
  const std::vector<hipEvent_t>* pool = nullptr;  // null: dry count
  size_t used = 0;
  hipError_t take(hipEvent_t* ev) {
    if (pool) {
      if (used >= pool->size()) return hipErrorInvalidValue;
      *ev = (*pool)[used];
    } else {
      *ev = nullptr;
    }
    ++used;
    return hipSuccess;
  }
  hipError_t record(hipEvent_t ev, hipStream_t st) { return pool ? hipEventRecord(ev, st) : hipSuccess; }
  hipError_t wait(hipStream_t st, hipEvent_t ev) { return pool ? hipStreamWaitEvent(st, ev, 0) : hipSuccess; }
  // an event recorded on `from` that `to` waits for
  hipError_t join(hipStream_t from, hipStream_t to) {
    hipEvent_t ev;
    hipError_t e = take(&ev);
    if (e == hipSuccess) e = record(ev, from);
    if (e == hipSuccess) e = wait(to, ev);
    return e;
  }
  hipError_t pass(const Group& g, int mode, const ChainDev* d_cd, const Tile* t, int n, int j, int k,
                  hipStream_t st) {
    return pool ? launch_lattice_pass(g.prec, g.ndim, g.cls, mode, d_cd, t, n, j, k, st) : hipSuccess;
  }
  hipError_t resident(const Group& g, const ChainDev* d_cd, const Tile* t, int n, int per_cu, hipStream_t st) {
    return pool ? launch_resident_group(g, d_cd, t, n, 1, per_cu, st) : hipSuccess;
  }
};

// One trajectory of every chain.  Per group: pass j = 0 (FIRST) over all
// tiles, then MIDDLE over the chains that still have passes after j and LAST
// over the chains whose final pass is j.  Chains are sorted by pass count, so
// each set is a contiguous range of the tile table.  Groups run on streams of
// their own, and the LAST launches of a group on a second stream: LAST(j) only
// waits for launch j-1 of its group, so it overlaps MIDDLE(j) of the other
// chains.  Captured once, the fork/join structure becomes graph edges.
static hipError_t round_plan(const std::vector<Group>& groups, const Tile* d_tiles, const ChainDev* d_cd,
                             const std::vector<hipStream_t>& side, RoundSink& sk, hipStream_t s) {
  hipError_t e;
  hipEvent_t fork;
  if ((e = sk.take(&fork)) != hipSuccess) return e;
  if ((e = sk.record(fork, s)) != hipSuccess) return e;
  // resident launches beside tiled groups leave half of each CU to their passes
  bool tiled = false;
  for (const Group& g : groups) tiled = tiled || g.cls >= 0;
  const int res_per_cu = tiled ? 1 : 2;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Group& g = groups[gi];
    hipStream_t gs = sk.pool ? side[gi] : nullptr;
    if ((e = sk.wait(gs, fork)) != hipSuccess) return e;
    const Tile* base = d_tiles + g.tile_off;
    if (g.cls < 0) {  // one launch runs the whole trajectory of every chain of the group
      if ((e = sk.resident(g, d_cd, base, g.tile_begin.back(), res_per_cu, gs)) != hipSuccess) return e;
      if ((e = sk.join(gs, s)) != hipSuccess) return e;
      continue;
    }
    if ((e = sk.pass(g, PASS_FIRST, d_cd, base, g.tile_begin.back(), 0, 0, gs)) != hipSuccess) return e;
    const int nc = (int)g.order.size();
    if (g.pair) {
      // Middle steps in pairs (1, 2), (3, 4), ...: launch k = 1 + (j - 1) / 2
      // runs the pair starting at odd j over the chains with passes after j
      // (chain order is descending pass count); a chain whose last middle step
      // is j (its last pass is j + 1) takes step j alone in the same launch.
      for (int j = 1; j < g.max_pass; j += 2) {
        const int k = 1 + (j - 1) / 2;
        int end = 0;
        while (end < nc && g.n_pass[end] - 1 > j) ++end;
        if (end > 0) {
          if ((e = sk.pass(g, PASS_PAIR, d_cd, base, g.tile_begin[end], j, k, gs)) != hipSuccess) return e;
        }
      }
    }
    for (int j = 1; !g.pair && j < g.max_pass; ++j) {
      int mid_end = 0;
      while (mid_end < nc && g.n_pass[mid_end] - 1 > j) ++mid_end;
      if (mid_end > 0) {
        if ((e = sk.pass(g, PASS_MIDDLE, d_cd, base, g.tile_begin[mid_end], j, j, gs)) != hipSuccess) return e;
      }
    }
    // the last pass of every chain of the group in one launch, each chain at
    // its own pass and buffers: no launch of the round waits on another stream
    if ((e = sk.pass(g, PASS_LAST, d_cd, base, g.tile_begin.back(), -1, g.pair ? 1 : 0, gs)) != hipSuccess)
      return e;
    if ((e = sk.join(gs, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t enqueue_round_plan(const std::vector<Group>& groups, const Tile* d_tiles, const ChainDev* d_cd,
                              const std::vector<hipStream_t>& side, const std::vector<hipEvent_t>& events,
                              hipStream_t s) {
  if (side.size() < groups.size()) return hipErrorInvalidValue;
  RoundSink sk;
  sk.pool = &events;
  return round_plan(groups, d_tiles, d_cd, side, sk, s);
}

size_t round_events_used(const std::vector<Group>& groups) {
  RoundSink sk;
  const std::vector<hipStream_t> none;
  round_plan(groups, nullptr, nullptr, none, sk, nullptr);
  return sk.used;
}

hipError_t Chains::enqueue_round(hipStream_t s) { return enqueue_round_plan(groups, d_tiles, d_cd, side, events, s); }

int Chains::advance(int32_t n_traj) {
  if (n_traj < 0) return set_error(IHMC_E_INVAL, "n_traj must be >= 0");
  for (int i = 0; i < n; ++i)
    if (base[i] + enqueued + n_traj > cd[i].cap)
      return set_error(IHMC_E_INVAL, "chain %d: %d trajectories exceed the capacity %d", i,
                       base[i] + enqueued + n_traj, cd[i].cap);
  hipStream_t s = ctx->stream;
  if (n_traj == 0) return IHMC_OK;
  bool all_resident = true;
  for (auto& g : groups) all_resident = all_resident && g.cls < 0;
  if (all_resident) {  // every chain in LDS: one launch per group runs all n_traj trajectories,
                       // the groups side by side on their own streams
    const bool fork = groups.size() > 1;
    if (fork) HIPCHK(hipEventRecord(events[0], s), "fork");
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      const Group& g = groups[gi];
      hipStream_t gs = fork ? side[gi] : s;
      if (fork) HIPCHK(hipStreamWaitEvent(gs, events[0], 0), "fork wait");
      HIPCHK(launch_resident_group(g, d_cd, d_tiles + g.tile_off, g.tile_begin.back(), n_traj, 2, gs),
             "resident launch");
      if (fork) {
        HIPCHK(hipEventRecord(events[1 + gi], gs), "join");
        HIPCHK(hipStreamWaitEvent(s, events[1 + gi], 0), "join wait");
      }
    }
    enqueued += n_traj;
    return IHMC_OK;
  }
  if (n_traj == 1 && !gexec) {
    HIPCHK(enqueue_round(s), "round launch");
  } else {
    if (!gexec) {
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
      hipError_t e = enqueue_round(s);
      hipGraph_t gr = nullptr;
      hipError_t e2 = hipStreamEndCapture(s, &gr);
      if (e != hipSuccess) return hip_fail(ctx, e, "capture round");
      if (e2 != hipSuccess) return hip_fail(ctx, e2, "end capture");
      graph = gr;
      HIPCHK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0), "graph instantiate");
    }
    for (int t = 0; t < n_traj; ++t) HIPCHK(hipGraphLaunch(gexec, s), "graph launch");
  }
  enqueued += n_traj;
  return IHMC_OK;
}

int Chains::checkpoint(int32_t i, void* buf, uint64_t* bytes) {
  if (i < 0 || i >= n) return set_error(IHMC_E_INVAL, "chain index %d out of range", i);
  return chain_checkpoint(ctx, cd[i], delta[i].empty() ? 0 : 1, buf, bytes);
}

int Chains::restore(int32_t i, const void* buf, uint64_t bytes) {
  if (i < 0 || i >= n) return set_error(IHMC_E_INVAL, "chain index %d out of range", i);
  int traj = 0;
  int rc = chain_restore(ctx, cd[i], delta[i].empty() ? 0 : 1, buf, bytes, &traj);
  if (rc) return rc;
  base[i] = traj - enqueued;
  return IHMC_OK;
}

int Chains::result(int32_t i, ihmc_result* out) {
  if (i < 0 || i >= n) return set_error(IHMC_E_INVAL, "chain index %d out of range", i);
  int rc = result_from_device(ctx, cd[i], d_cd, i, out);
  if (rc || delta[i].empty()) return rc;
  // a translated shifted-form chain: its field and action in its own coordinates
  const int64_t done = std::min<int64_t>(out->n_traj_done, cd[i].cap);
  for (int64_t t = 0; t < done; ++t) {
    if (out->H_old) out->H_old[t] += s_offset[i];
    if (out->H_new) out->H_new[t] += s_offset[i];
  }
  if (out->psi_final)
    for (int64_t k = 0; k < cd[i].N; ++k) out->psi_final[k] -= delta[i][(size_t)k];
  return IHMC_OK;
}

// Series and summary of chain ci of a device chain table (shared by the lattice
// and dense runtimes).
int result_from_device(ihmc_ctx* ctx, const ChainDev& c, const ChainDev* d_cd, int ci, ihmc_result* out) {
  if (!out) return set_error(IHMC_E_INVAL, "out is NULL");
  hipStream_t s = ctx->stream;
  HIPCHK(hipStreamSynchronize(s), "sync");
  ChainState st;
  HIPCHK(hipMemcpy(&st, c.st, sizeof st, hipMemcpyDeviceToHost), "state download");
  const int done = std::min(st.traj, c.cap);
  std::vector<TrajRecord> rec((size_t)std::max(done, 1));
  if (done > 0) HIPCHK(hipMemcpy(rec.data(), c.rec, sizeof(TrajRecord) * done, hipMemcpyDeviceToHost), "records");
  for (int t = 0; t < done; ++t) {
    const TrajRecord& r = rec[t];
    if (out->dH) out->dH[t] = r.dH;
    if (out->H_old) out->H_old[t] = r.H_old;
    if (out->H_new) out->H_new[t] = r.H_new;
    if (out->m) out->m[t] = r.m;
    if (out->abs_m) out->abs_m[t] = r.abs_m;
    if (out->m2c) out->m2c[t] = r.m2c;
    if (out->beta_eps) out->beta_eps[t] = r.beta_eps;
    if (out->accepted) out->accepted[t] = (r.flags & REC_ACCEPT) ? 1 : 0;
    if (out->flipped) out->flipped[t] = (r.flags & REC_FLIP) ? 1 : 0;
  }
  out->n_traj_done = st.traj;
  const int64_t counted = std::max(0, st.traj - c.n_therm);  // trajectories past thermalisation
  out->acceptance = counted ? (double)st.n_acc / (double)counted : 0.0;
  const int64_t nf = counted - st.n_nonfinite;
  out->mean_exp_minus_dH = nf > 0 ? st.sum_exp_mdh / (double)nf : 0.0;
  out->n_nonfinite = st.n_nonfinite;
  out->cg_iterations = st.n_cg;
  if (out->psi_final) {
    double* t = (double*)ctx->arena.alloc(8 * (uint64_t)c.N);
    if (!t) return set_error(IHMC_E_NOMEM, "arena exhausted (export)");
    hipError_t e0 = launch_export_psi(d_cd, ci, t, c.N, c.precision, s);
    hipError_t e = e0 == hipSuccess ? hipMemcpyAsync(out->psi_final, t, 8 * c.N, hipMemcpyDeviceToHost, s) : e0;
    hipError_t e2 = hipStreamSynchronize(s);
    ctx->arena.release(t);
    if (e != hipSuccess) return hip_fail(ctx, e, "psi export");
    if (e2 != hipSuccess) return hip_fail(ctx, e2, "psi export sync");
  }
  return IHMC_OK;
}

// ------------------------------------------------------ checkpoint / resume ---
//
// A chain's state between trajectories: the accepted field (buffer `cur`),
// ChainState (S in fixed point, estimator sums, sign, counters, next
// trajectory index) and the records so far.  Every random number is a Philox
// draw at counters that name the trajectory, so this is all the state there is.

namespace {
constexpr char kCkptMagic[8] = {'I', 'H', 'M', 'C', 'C', 'K', 'P', 'T'};
constexpr uint32_t kCkptVersion = 2;

struct CkptHeader {
  char magic[8];
  uint32_t version, header_bytes;
  // identity of the chain: everything its trajectories depend on
  int32_t ndim, L0, L1, L2;
  int64_t N, NP;
  int32_t precision, n_pass, integrator, flip_every;
  uint32_t chain_id, seed_lo, seed_hi;
  int32_t h_kind, form, pad0;
  double C, sqJ, Jp, b0, hp0, eps, c_m, c_e, c_v;
  uint64_t field_hash;  // FNV-1a of the per-site h' in site order (0 without one)
  uint64_t variant;     // path-specific form of the force (dense: limb products)
  // state
  ChainState st;
  int32_t n_rec, pad;
};

void fill_identity(const ChainDev& c, uint64_t field_hash, uint64_t variant, CkptHeader& h) {
  h.ndim = c.ndim;
  h.L0 = c.L0;
  h.L1 = c.L1;
  h.L2 = c.L2;
  h.N = c.N;
  h.NP = c.NP;
  h.precision = c.precision;
  h.n_pass = c.n_pass;
  h.integrator = c.integrator;
  h.flip_every = c.flip_every;
  h.chain_id = c.chain_id;
  h.seed_lo = c.seed_lo;
  h.seed_hi = c.seed_hi;
  h.h_kind = c.h_kind;
  h.form = c.form;
  h.C = c.C;
  h.sqJ = c.sqJ;
  h.Jp = c.Jp;
  h.b0 = c.b0;
  h.hp0 = c.hp0;
  h.eps = c.eps;
  h.c_m = c.c_m;
  h.c_e = c.c_e;
  h.c_v = c.c_v;
  h.field_hash = field_hash;
  h.variant = variant;
}

// FNV-1a over the per-site FP64 h' of the chain (device array of NP values in
// the stored layout; the padding of the rows is skipped).
int field_hash(ihmc_ctx* ctx, const ChainDev& c, hipStream_t s, uint64_t* out) {
  *out = 0;
  if (c.h_kind != 2 || !c.hp) return IHMC_OK;
  std::vector<double> hp((size_t)c.NP);
  HIPCHK(hipMemcpyAsync(hp.data(), c.hp, 8 * (size_t)c.NP, hipMemcpyDeviceToHost, s), "field download");
  HIPCHK(hipStreamSynchronize(s), "sync");
  std::vector<double> logical((size_t)c.N);
  for (int64_t i = 0; i < c.N; ++i) logical[(size_t)i] = hp[(size_t)stored_index(c, i)];
  *out = field_hash_host(logical.data(), c.N);
  return IHMC_OK;
}

uint64_t checkpoint_bytes(const ChainDev& c, int n_rec) {
  return sizeof(CkptHeader) + (uint64_t)c.NP * (uint64_t)c.precision + (uint64_t)n_rec * sizeof(TrajRecord);
}
}  // namespace

uint64_t field_hash_host(const double* hp, int64_t n) {
  uint64_t h = 1469598103934665603ull;
  const unsigned char* b = (const unsigned char*)hp;
  for (size_t k = 0; k < (size_t)n * 8; ++k) h = (h ^ b[k]) * 1099511628211ull;
  return h;
}

uint64_t chain_checkpoint_max_bytes(const ChainDev& c) { return checkpoint_bytes(c, std::max(0, c.cap)); }

int chain_checkpoint(ihmc_ctx* ctx, const ChainDev& c, uint64_t variant, void* buf, uint64_t* bytes, hipStream_t s) {
  if (!bytes) return set_error(IHMC_E_INVAL, "bytes is NULL");
  if (!s) s = ctx->stream;
  HIPCHK(hipStreamSynchronize(s), "sync");
  ChainState st;
  HIPCHK(hipMemcpyAsync(&st, c.st, sizeof st, hipMemcpyDeviceToHost, s), "state download");
  HIPCHK(hipStreamSynchronize(s), "sync");
  const int n_rec = std::max(0, std::min(st.traj, c.cap));
  const uint64_t field = (uint64_t)c.NP * (uint64_t)c.precision;
  const uint64_t need = checkpoint_bytes(c, n_rec);
  if (!buf) {
    *bytes = need;
    return IHMC_OK;
  }
  if (*bytes < need) {
    const uint64_t have = *bytes;
    *bytes = need;
    return set_error(IHMC_E_INVAL, "checkpoint buffer of %llu bytes, %llu needed", (unsigned long long)have,
                     (unsigned long long)need);
  }
  CkptHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, kCkptMagic, 8);
  h.version = kCkptVersion;
  h.header_bytes = sizeof h;
  uint64_t fh = 0;
  int rc = field_hash(ctx, c, s, &fh);
  if (rc) return rc;
  fill_identity(c, fh, variant, h);
  h.st = st;
  h.n_rec = n_rec;
  char* out = (char*)buf;
  std::memcpy(out, &h, sizeof h);
  HIPCHK(hipMemcpyAsync(out + sizeof h, (const char*)c.psi + (uint64_t)st.cur * field, field, hipMemcpyDeviceToHost, s),
         "field download");
  if (n_rec)
    HIPCHK(hipMemcpyAsync(out + sizeof h + field, c.rec, sizeof(TrajRecord) * (size_t)n_rec, hipMemcpyDeviceToHost, s),
           "records download");
  HIPCHK(hipStreamSynchronize(s), "sync");
  *bytes = need;
  return IHMC_OK;
}

int chain_checkpoint_host(const ChainDev& c, uint64_t fh, const ChainState& st_in, const double* psi,
                          const TrajRecord* rec, int n_rec, std::vector<char>& out) {
  const uint64_t field = (uint64_t)c.NP * (uint64_t)c.precision;
  out.assign(checkpoint_bytes(c, n_rec), 0);
  CkptHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, kCkptMagic, 8);
  h.version = kCkptVersion;
  h.header_bytes = sizeof h;
  fill_identity(c, fh, 0, h);
  h.st = st_in;
  // the field is given with its sign applied: it is stored as is, with sign +1
  // (every pass reads the stored field times the sign, and negation is exact)
  h.st.cur = 0;
  h.st.sign = 1;
  h.st.done = 0u;
  h.st.bad = 0u;
  h.n_rec = n_rec;
  std::memcpy(out.data(), &h, sizeof h);
  char* f = out.data() + sizeof h;
  for (int64_t i = 0; i < c.N; ++i) {
    const int64_t k = stored_index(c, i);
    if (c.precision == 4) {
      const float v = (float)psi[i];
      std::memcpy(f + 4 * k, &v, 4);
    } else {
      std::memcpy(f + 8 * k, &psi[i], 8);
    }
  }
  if (n_rec) std::memcpy(out.data() + sizeof h + field, rec, sizeof(TrajRecord) * (size_t)n_rec);
  return IHMC_OK;
}

int chain_restore(ihmc_ctx* ctx, const ChainDev& c, uint64_t variant, const void* buf, uint64_t bytes, int* traj,
                  hipStream_t s) {
  if (!buf) return set_error(IHMC_E_INVAL, "buf is NULL");
  if (bytes < sizeof(CkptHeader)) return set_error(IHMC_E_INVAL, "not a checkpoint (%llu bytes)", (unsigned long long)bytes);
  if (!s) s = ctx->stream;
  CkptHeader h;
  std::memcpy(&h, buf, sizeof h);
  if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != kCkptVersion || h.header_bytes != sizeof h)
    return set_error(IHMC_E_INVAL, "not a checkpoint of this library version");
  uint64_t fh = 0;
  HIPCHK(hipStreamSynchronize(s), "sync");
  int rc = field_hash(ctx, c, s, &fh);
  if (rc) return rc;
  CkptHeader mine;
  std::memset(&mine, 0, sizeof mine);
  fill_identity(c, fh, variant, mine);
  // compare the identity fields (the span between the version words and the state)
  const size_t id0 = offsetof(CkptHeader, ndim), id1 = offsetof(CkptHeader, st);
  if (std::memcmp((const char*)&h + id0, (const char*)&mine + id0, id1 - id0) != 0)
    return set_error(IHMC_E_INVAL, "checkpoint of a chain with other parameters");
  const ChainState& st = h.st;
  if (st.traj < 0 || st.cur < 0 || st.cur >= LAT_BUFFERS || (st.sign != 1 && st.sign != -1) || h.n_rec != st.traj)
    return set_error(IHMC_E_INVAL, "checkpoint state is inconsistent");
  if (st.traj > c.cap)
    return set_error(IHMC_E_INVAL, "checkpoint after %d trajectories, the chain's capacity is %d", st.traj, c.cap);
  const uint64_t field = (uint64_t)c.NP * (uint64_t)c.precision;
  const uint64_t need = checkpoint_bytes(c, h.n_rec);
  if (bytes != need)
    return set_error(IHMC_E_INVAL, "checkpoint of %llu bytes, %llu expected", (unsigned long long)bytes,
                     (unsigned long long)need);
  ChainState ns = st;
  ns.cur = 0;  // the field goes to buffer 0
  ns.done = 0u;
  ns.bad = 0u;
  const char* in = (const char*)buf;
  HIPCHK(hipMemcpyAsync(c.psi, in + sizeof h, field, hipMemcpyHostToDevice, s), "field upload");
  if (h.n_rec)
    HIPCHK(hipMemcpyAsync(c.rec, in + sizeof h + field, sizeof(TrajRecord) * (size_t)h.n_rec, hipMemcpyHostToDevice, s),
           "records upload");
  HIPCHK(hipMemcpyAsync(c.st, &ns, sizeof ns, hipMemcpyHostToDevice, s), "state upload");
  HIPCHK(hipStreamSynchronize(s), "sync");
  *traj = st.traj;
  return IHMC_OK;
}

}  // namespace ihmc

// ========================================================== C ABI: chains ===



static int make_chains(ihmc_ctx* ctx, int32_t n, const ihmc_lattice* lats, const ihmc_run* runs, int flags,
                       Chains** out) {
  if (n < 1 || !lats || !runs) return set_error(IHMC_E_INVAL, "need n >= 1 chains with descriptors");
  Chains* c = new (std::nothrow) Chains();
  if (!c) return set_error(IHMC_E_NOMEM, "host allocation failed");
  c->ctx = ctx;
  int rc = c->build(n, lats, runs, flags);
  if (rc) {
    hipStreamSynchronize(ctx->stream);
    delete c;
    return rc;
  }
  *out = c;
  return IHMC_OK;
}

extern "C" int ihmc_chains_create(ihmc_ctx* ctx, int32_t n, const ihmc_lattice* lats, const ihmc_run* runs,
                                  ihmc_chains** out) {
  CTX_OK(ctx);
  if (!out) return set_error(IHMC_E_INVAL, "out is NULL");
  Chains* c = nullptr;
  int rc = make_chains(ctx, n, lats, runs, 0, &c);
  *out = (ihmc_chains*)c;
  return rc;
}

extern "C" int ihmc_chains_advance(ihmc_chains* ch, int32_t n_traj) {
  if (!ch) return set_error(IHMC_E_INVAL, "chains is NULL");
  Chains* c = (Chains*)ch;
  CTX_OK(c->ctx);
  return c->advance(n_traj);
}

extern "C" int ihmc_chains_result(ihmc_chains* ch, int32_t i, ihmc_result* out) {
  if (!ch) return set_error(IHMC_E_INVAL, "chains is NULL");
  Chains* c = (Chains*)ch;
  CTX_OK(c->ctx);
  return c->result(i, out);
}

extern "C" int ihmc_chains_checkpoint(ihmc_chains* ch, int32_t i, void* buf, uint64_t* bytes) {
  if (!ch) return set_error(IHMC_E_INVAL, "chains is NULL");
  Chains* c = (Chains*)ch;
  CTX_OK(c->ctx);
  return c->checkpoint(i, buf, bytes);
}

extern "C" int ihmc_chains_restore(ihmc_chains* ch, int32_t i, const void* buf, uint64_t bytes) {
  if (!ch) return set_error(IHMC_E_INVAL, "chains is NULL");
  Chains* c = (Chains*)ch;
  CTX_OK(c->ctx);
  return c->restore(i, buf, bytes);
}

extern "C" int ihmc_chains_destroy(ihmc_chains* ch) {
  if (!ch) return IHMC_OK;
  Chains* c = (Chains*)ch;
  hipSetDevice(c->ctx->device);
  hipStreamSynchronize(c->ctx->stream);
  delete c;
  return IHMC_OK;
}

extern "C" int ihmc_run_batch(ihmc_ctx* ctx, int32_t n, const ihmc_lattice* lats, const ihmc_run* runs,
                              ihmc_result* outs) {
  CTX_OK(ctx);
  if (!outs) return set_error(IHMC_E_INVAL, "outs is NULL");
  Chains* c = nullptr;
  int rc = make_chains(ctx, n, lats, runs, 0, &c);
  if (rc) return rc;
  int max_traj = 0;
  bool uniform = true;
  for (int i = 0; i < n; ++i) {
    max_traj = std::max(max_traj, runs[i].n_traj);
    uniform = uniform && runs[i].n_traj == runs[0].n_traj;
  }
  if (!uniform) {
    delete c;
    return set_error(IHMC_E_UNSUPPORTED, "ihmc_run_batch: chains must share n_traj");
  }
  rc = c->advance(max_traj);
  for (int i = 0; rc == IHMC_OK && i < n; ++i) rc = c->result(i, &outs[i]);
  hipStreamSynchronize(ctx->stream);
  delete c;
  return rc;
}

extern "C" int ihmc_run_lattice(ihmc_ctx* ctx, const ihmc_lattice* lat, const ihmc_run* run, ihmc_result* out) {
  return ihmc_run_batch(ctx, 1, lat, run, out);
}

// ===================================================== C ABI: diagnostics ===

static ihmc_run diag_run(int32_t precision) {
  ihmc_run r;
  std::memset(&r, 0, sizeof r);
  r.n_md = 1;
  r.n_traj = 1;
  r.traj_len = 1.0;
  r.precision = precision;
  return r;
}

extern "C" int ihmc_force(ihmc_ctx* ctx, const ihmc_lattice* lat, int32_t precision, const double* psi, double* F) {
  CTX_OK(ctx);
  if (!lat || !psi || !F) return set_error(IHMC_E_INVAL, "NULL argument");
  ihmc_run r = diag_run(precision);
  r.psi0 = psi;
  Chains* c = nullptr;
  int rc = make_chains(ctx, 1, lat, &r, BUILD_TILED, &c);  // the force pass is a tiled-kernel mode
  if (rc) return rc;
  hipStream_t s = ctx->stream;
  const Group& g = c->groups[0];
  hipError_t e = launch_lattice_pass(g.prec, g.ndim, g.cls, PASS_FORCE, c->d_cd, c->d_tiles, g.tile_begin.back(), 0, 0, s);
  const int64_t N = c->cd[0].N;
  double* t = (double*)ctx->arena.alloc(8 * (uint64_t)N);
  if (e == hipSuccess && t) {
    if (precision == 4) k_export<float><<<nblk(N), 256, 0, s>>>(c->d_cd, 0, t, (const float*)c->cd[0].p);
    else k_export<double><<<nblk(N), 256, 0, s>>>(c->d_cd, 0, t, (const double*)c->cd[0].p);
    e = hipMemcpyAsync(F, t, 8 * N, hipMemcpyDeviceToHost, s);
  }
  hipError_t e2 = hipStreamSynchronize(s);
  if (t) ctx->arena.release(t);
  delete c;
  if (!t) return set_error(IHMC_E_NOMEM, "arena exhausted");
  if (e != hipSuccess) return hip_fail(ctx, e, "force");
  if (e2 != hipSuccess) return hip_fail(ctx, e2, "force sync");
  return IHMC_OK;
}

extern "C" int ihmc_action(ihmc_ctx* ctx, const ihmc_lattice* lat, int32_t precision, const double* psi,
                           double* out) {
  CTX_OK(ctx);
  if (!lat || !psi || !out) return set_error(IHMC_E_INVAL, "NULL argument");
  ihmc_run r = diag_run(precision);
  r.psi0 = psi;
  Chains* c = nullptr;
  int rc = make_chains(ctx, 1, lat, &r, 0, &c);
  if (rc) return rc;
  ChainState st;
  ChainDev cdv;
  hipError_t e = hipMemcpy(&st, c->cd[0].st, sizeof st, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&cdv, c->d_cd, sizeof cdv, hipMemcpyDeviceToHost);
  delete c;
  if (e != hipSuccess) return hip_fail(ctx, e, "action download");
  const double N = (double)cdv.N;
  out[0] = fixed_to_double(u128{st.S_lo, st.S_hi});
  out[1] = (st.sum_psi / cdv.sqJ - cdv.c_m / cdv.Jp) / N;
  out[2] = std::fabs(out[1]);
  out[3] = out[1] * out[1] - cdv.c_v / (N * N * cdv.Jp);
  out[4] = 0.5 * cdv.C * cdv.Jp + cdv.c_e / (2.0 * N * cdv.Jp) - st.sum_psih / (2.0 * N * cdv.sqJ) -
           cdv.sqJ / (2.0 * N) * st.sum_ut;
  return IHMC_OK;
}

extern "C" int ihmc_integrate(ihmc_ctx* ctx, const ihmc_lattice* lat, const ihmc_run* run, double* psi, double* p) {
  CTX_OK(ctx);
  if (!lat || !run || !psi || !p) return set_error(IHMC_E_INVAL, "NULL argument");
  ihmc_run r = *run;
  r.n_traj = 1;
  r.psi0 = psi;
  r.flip_every = 0;
  static const uint8_t one = 1;
  r.replay_accept = &one;
  Chains* c = nullptr;
  int rc = make_chains(ctx, 1, lat, &r, BUILD_P_GIVEN | BUILD_WRITE_P, &c);
  if (rc) return rc;
  hipStream_t s = ctx->stream;
  const ChainDev& cdh = c->cd[0];
  const int64_t N = cdh.N;
  double* t = (double*)ctx->arena.alloc(8 * (uint64_t)N);
  hipError_t e = hipSuccess;
  if (t) {
    e = hipMemcpyAsync(t, p, 8 * N, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      if (cdh.precision == 4) k_import<float><<<nblk(N), 256, 0, s>>>(c->d_cd, 0, (float*)cdh.p, t);
      else k_import<double><<<nblk(N), 256, 0, s>>>(c->d_cd, 0, (double*)cdh.p, t);
      e = c->enqueue_round(s);
    }
    if (e == hipSuccess) {
      if (cdh.precision == 4) k_export_psi<float><<<nblk(N), 256, 0, s>>>(c->d_cd, 0, t);
      else k_export_psi<double><<<nblk(N), 256, 0, s>>>(c->d_cd, 0, t);
      e = hipMemcpyAsync(psi, t, 8 * N, hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && !c->delta[0].empty())  // a translated shifted-form chain
      for (int64_t k = 0; k < N; ++k) psi[k] -= c->delta[0][(size_t)k];
    if (e == hipSuccess) {
      if (cdh.precision == 4) k_export<float><<<nblk(N), 256, 0, s>>>(c->d_cd, 0, t, (const float*)cdh.p);
      else k_export<double><<<nblk(N), 256, 0, s>>>(c->d_cd, 0, t, (const double*)cdh.p);
      e = hipMemcpyAsync(p, t, 8 * N, hipMemcpyDeviceToHost, s);
    }
  }
  hipError_t e2 = hipStreamSynchronize(s);
  if (t) ctx->arena.release(t);
  delete c;
  if (!t) return set_error(IHMC_E_NOMEM, "arena exhausted");
  if (e != hipSuccess) return hip_fail(ctx, e, "integrate");
  if (e2 != hipSuccess) return hip_fail(ctx, e2, "integrate sync");
  return IHMC_OK;
}

extern "C" int ihmc_hamiltonian(ihmc_ctx* ctx, const ihmc_lattice* lat, int32_t precision, const double* psi,
                                const double* p, double* H) {
  CTX_OK(ctx);
  if (!lat || !psi || !p || !H) return set_error(IHMC_E_INVAL, "NULL argument");
  *H = NAN;
  // H_old of a trajectory whose first pass reads the given momenta: the
  // kinetic sum of that pass plus S(psi) of the set-up measurement, added in
  // exact fixed point by the closing block.  The trajectory itself is made
  // negligibly short (its kicks and drifts round away), so no term of the
  // final state can flag the record unless the given state already does.
  ihmc_run r = diag_run(precision);
  r.psi0 = psi;
  r.traj_len = 1e-300;
  static const uint8_t one = 1;
  r.replay_accept = &one;
  Chains* c = nullptr;
  int rc = make_chains(ctx, 1, lat, &r, BUILD_P_GIVEN, &c);
  if (rc) return rc;
  hipStream_t s = ctx->stream;
  const ChainDev& cdh = c->cd[0];
  const int64_t N = cdh.N;
  double* t = (double*)ctx->arena.alloc(8 * (uint64_t)N);
  hipError_t e = t ? hipMemcpyAsync(t, p, 8 * N, hipMemcpyHostToDevice, s) : hipSuccess;
  if (t && e == hipSuccess) {
    if (cdh.precision == 4) k_import<float><<<nblk(N), 256, 0, s>>>(c->d_cd, 0, (float*)cdh.p, t);
    else k_import<double><<<nblk(N), 256, 0, s>>>(c->d_cd, 0, (double*)cdh.p, t);
    e = c->enqueue_round(s);
  }
  TrajRecord rec;
  std::memset(&rec, 0, sizeof rec);
  if (t && e == hipSuccess) e = hipMemcpyAsync(&rec, cdh.rec, sizeof rec, hipMemcpyDeviceToHost, s);
  hipError_t e2 = hipStreamSynchronize(s);
  if (t) ctx->arena.release(t);
  delete c;
  if (!t) return set_error(IHMC_E_NOMEM, "arena exhausted");
  if (e != hipSuccess) return hip_fail(ctx, e, "hamiltonian");
  if (e2 != hipSuccess) return hip_fail(ctx, e2, "hamiltonian sync");
  if (rec.flags & REC_NONFINITE)
    return set_error(IHMC_E_INVAL, "a term of H(psi, p) is non-finite or too large for the exact sums");
  *H = rec.H_old;
  return IHMC_OK;
}

extern "C" int ihmc_plan_events(int32_t n, const ihmc_lattice* lats, const ihmc_run* runs, int32_t fuse_steps,
                                int64_t resident_sites, int64_t* taken, int64_t* reserved) {
  if (n < 1 || !lats || !runs || !taken || !reserved) return set_error(IHMC_E_INVAL, "bad arguments");
  std::vector<ChainDev> cd((size_t)n);
  for (int i = 0; i < n; ++i) {
    int rc = validate(lats[i], runs[i], i);
    if (rc) return rc;
    const ihmc_lattice& l = lats[i];
    const bool site_field = !(l.h_len == 0 || l.h_len == 1);
    const int64_t fit = resident_max_sites(runs[i].precision, site_field);
    const int64_t lim = resident_sites < 0 ? fit : std::min(fit, resident_sites);
    const int cls = runs[i].form == FORM_PHI ? RESIDENT_PHI_CLASS
                    : lattice_sites(l) <= lim ? RESIDENT_CLASS
                                              : tile_class(l.ndim, l.L[0], l.ndim == 3 ? l.L[2] : 1);
    describe_chain(l, runs[i], 0, cls, cd[i]);
  }
  std::vector<int> members((size_t)n);
  for (int i = 0; i < n; ++i) members[i] = i;
  std::vector<Group> groups;
  std::vector<Tile> tiles;
  plan_groups(cd, members, groups, tiles, fuse_steps != 0);
  *taken = (int64_t)round_events_used(groups);
  *reserved = (int64_t)round_events(groups);
  return IHMC_OK;
}

extern "C" int ihmc_fixed_point(int64_t n, const double* x, uint64_t* out, int32_t* ok) {
  if (n < 0 || (n > 0 && (!x || !out || !ok))) return set_error(IHMC_E_INVAL, "bad arguments");
  for (int64_t i = 0; i < n; ++i) {
    u128 v;
    ok[i] = to_fixed_wide(x[i], v) ? 1 : 0;
    out[2 * i] = v.lo;
    out[2 * i + 1] = v.hi;
  }
  return IHMC_OK;
}

extern "C" int ihmc_philox_normals(ihmc_ctx* ctx, uint64_t seed, uint64_t chain_id, uint32_t traj, uint32_t tag,
                                   int32_t precision, int64_t n, double* out) {
  CTX_OK(ctx);
  if (n < 0 || (n > 0 && !out)) return set_error(IHMC_E_INVAL, "bad output");
  if (precision != 4 && precision != 8) return set_error(IHMC_E_INVAL, "precision must be 4 or 8");
  if (n == 0) return IHMC_OK;
  ChainDev cdv;
  std::memset(&cdv, 0, sizeof cdv);
  cdv.seed_lo = (uint32_t)seed;
  cdv.seed_hi = (uint32_t)(seed >> 32);
  cdv.chain_id = (uint32_t)chain_id;
  double* t = (double*)ctx->arena.alloc(8 * (uint64_t)n);
  if (!t) return set_error(IHMC_E_NOMEM, "arena exhausted");
  hipStream_t s = ctx->stream;
  const int64_t pairs = (n + 1) / 2;
  if (precision == 4) k_philox_normals<float><<<nblk(pairs), 256, 0, s>>>(cdv, traj, tag, n, t);
  else k_philox_normals<double><<<nblk(pairs), 256, 0, s>>>(cdv, traj, tag, n, t);
  hipError_t e = hipMemcpyAsync(out, t, 8 * n, hipMemcpyDeviceToHost, s);
  hipError_t e2 = hipStreamSynchronize(s);
  ctx->arena.release(t);
  if (e != hipSuccess) return hip_fail(ctx, e, "normals");
  if (e2 != hipSuccess) return hip_fail(ctx, e2, "normals sync");
  return IHMC_OK;
}

extern "C" int ihmc_philox_words(ihmc_ctx* ctx, int64_t n, const uint32_t* ctr, const uint32_t* key,
                                 uint32_t* out) {
  CTX_OK(ctx);
  if (n < 0 || (n > 0 && (!ctr || !key || !out))) return set_error(IHMC_E_INVAL, "bad arguments");
  if (n == 0) return IHMC_OK;
  uint32_t* d = (uint32_t*)ctx->arena.alloc(40 * (uint64_t)n);
  if (!d) return set_error(IHMC_E_NOMEM, "arena exhausted");
  hipStream_t s = ctx->stream;
  uint32_t *dc = d, *dk = d + 4 * n, *dout = d + 6 * n;
  hipError_t e = hipMemcpyAsync(dc, ctr, 16 * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dk, key, 8 * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    k_philox_words<<<nblk(n), 256, 0, s>>>(n, dc, dk, dout);
    e = hipMemcpyAsync(out, dout, 16 * n, hipMemcpyDeviceToHost, s);
  }
  hipError_t e2 = hipStreamSynchronize(s);
  ctx->arena.release(d);
  if (e != hipSuccess) return hip_fail(ctx, e, "philox");
  if (e2 != hipSuccess) return hip_fail(ctx, e2, "philox sync");
  return IHMC_OK;
}

// ======================================================== C ABI: measurement ===

extern "C" int ihmc_chains_groups(ihmc_chains* ch, int32_t* n_groups) {
  if (!ch || !n_groups) return set_error(IHMC_E_INVAL, "NULL argument");
  *n_groups = (int32_t)((Chains*)ch)->groups.size();
  return IHMC_OK;
}

extern "C" int ihmc_chains_group_info(ihmc_chains* ch, int32_t group, int64_t* out) {
  if (!ch || !out) return set_error(IHMC_E_INVAL, "NULL argument");
  Chains* c = (Chains*)ch;
  if (group < 0 || group >= (int32_t)c->groups.size()) return set_error(IHMC_E_INVAL, "group out of range");
  const Group& g = c->groups[group];
  int64_t sites = 0;
  for (int ci : g.order) sites += c->cd[ci].N;
  out[0] = g.prec;
  out[1] = g.ndim;
  out[2] = g.cls;
  out[3] = (int64_t)g.order.size();
  out[4] = sites;
  out[5] = g.tile_begin.back();
  return IHMC_OK;
}

extern "C" int ihmc_chains_group_chains(ihmc_chains* ch, int32_t group, int32_t* chain_idx) {
  if (!ch || !chain_idx) return set_error(IHMC_E_INVAL, "NULL argument");
  Chains* c = (Chains*)ch;
  if (group < 0 || group >= (int32_t)c->groups.size()) return set_error(IHMC_E_INVAL, "group out of range");
  const Group& g = c->groups[group];
  for (size_t i = 0; i < g.order.size(); ++i) chain_idx[i] = g.order[i];
  return IHMC_OK;
}

extern "C" int ihmc_chains_time_pass(ihmc_chains* ch, int32_t group, int32_t mode, int32_t reps, double* avg_us,
                                     int64_t* sites, int32_t* ndim, int32_t* precision) {
  if (!ch) return set_error(IHMC_E_INVAL, "chains is NULL");
  Chains* c = (Chains*)ch;
  ihmc_ctx* ctx = c->ctx;
  CTX_OK(ctx);
  if (group < 0 || group >= (int32_t)c->groups.size()) return set_error(IHMC_E_INVAL, "group out of range");
  if (mode != PASS_FIRST && mode != PASS_MIDDLE && mode != PASS_LAST && mode != PASS_PAIR)
    return set_error(IHMC_E_INVAL, "only FIRST, MIDDLE, LAST and PAIR passes can be timed");
  if (reps < 1) return set_error(IHMC_E_INVAL, "reps must be >= 1");
  const Group& g = c->groups[group];
  if (g.cls < 0)
    return set_error(IHMC_E_UNSUPPORTED, "group %d runs LDS-resident whole trajectories, not passes", group);
  if (mode == PASS_PAIR && g.ndim != 2)
    return set_error(IHMC_E_UNSUPPORTED, "group %d: two-step launches are 2D only", group);
  for (int ci : g.order) {
    if (mode == PASS_MIDDLE && c->cd[ci].n_pass < 3)
      return set_error(IHMC_E_INVAL, "chain %d has no middle pass", ci);
    if (mode == PASS_PAIR && c->cd[ci].n_pass < 4)
      return set_error(IHMC_E_INVAL, "chain %d has fewer than two middle steps", ci);
  }
  int64_t nsite = 0;
  for (int ci : g.order) nsite += c->cd[ci].N;
  hipStream_t s = ctx->stream;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0), "event");
  HIPCHK(hipEventCreate(&e1), "event");
  hipError_t e = launch_lattice_pass(g.prec, g.ndim, g.cls, mode, c->d_cd, c->d_tiles + g.tile_off, g.tile_begin.back(), 1, 1, s);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int r = 0; e == hipSuccess && r < reps; ++r)
    e = launch_lattice_pass(g.prec, g.ndim, g.cls, mode, c->d_cd, c->d_tiles + g.tile_off, g.tile_begin.back(), 1, 1, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(ctx, e, "time pass");
  if (avg_us) *avg_us = 1000.0 * ms / reps;
  if (sites) *sites = nsite;
  if (ndim) *ndim = g.ndim;
  if (precision) *precision = g.prec;
  return IHMC_OK;
}

// Plain streaming copy, one 16-byte vector per thread over a full grid (the
// fastest of the plain forms measured on this part: a grid-stride loop over a
// fixed grid reaches about 25 % less): the achievable-bandwidth reference for
// the roofline and the calibration of the memory counters.
__global__ __launch_bounds__(256) void k_copy_stream(const float4* __restrict__ src, float4* __restrict__ dst,
                                                     int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

extern "C" int ihmc_copy_bandwidth(ihmc_ctx* ctx, uint64_t bytes, int32_t reps, double* avg_us) {
  CTX_OK(ctx);
  if (bytes < 4096 || reps < 1) return set_error(IHMC_E_INVAL, "need bytes >= 4096 and reps >= 1");
  bytes &= ~(uint64_t)15;
  void* a = ctx->arena.alloc(bytes);
  void* b = ctx->arena.alloc(bytes);
  if (!a || !b) {
    ctx->arena.release(a);
    ctx->arena.release(b);
    return set_error(IHMC_E_NOMEM, "arena exhausted (copy buffers)");
  }
  hipStream_t s = ctx->stream;
  const int64_t n = (int64_t)(bytes / 16);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0), "event");
  HIPCHK(hipEventCreate(&e1), "event");
  if (n > (int64_t)256 * 0x7fffffff) return set_error(IHMC_E_INVAL, "copy too large");
  const unsigned grid = (unsigned)((n + 255) / 256);
  hipError_t e = hipMemsetAsync(a, 0, bytes, s);
  if (e == hipSuccess) {
    k_copy_stream<<<grid, 256, 0, s>>>((const float4*)a, (float4*)b, n);
    e = hipEventRecord(e0, s);
  }
  for (int r = 0; e == hipSuccess && r < reps; ++r) {
    k_copy_stream<<<grid, 256, 0, s>>>((const float4*)a, (float4*)b, n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  ctx->arena.release(a);
  ctx->arena.release(b);
  if (e != hipSuccess) return hip_fail(ctx, e, "copy bandwidth");
  if (avg_us) *avg_us = 1000.0 * ms / reps;
  return IHMC_OK;
}

namespace ihmc {
hipError_t launch_init_psi(const ChainDev* d_cd, int ci, const double* psi0, int64_t N, int precision, hipStream_t s,
                           const double* shift) {
  if (precision == 4) k_init_psi<float><<<nblk(N), 256, 0, s>>>(d_cd, ci, psi0, shift);
  else k_init_psi<double><<<nblk(N), 256, 0, s>>>(d_cd, ci, psi0, shift);
  return hipGetLastError();
}
hipError_t launch_scale(double* x, int64_t n, double by, hipStream_t s) {
  k_scale<<<nblk(n), 256, 0, s>>>(x, n, by);
  return hipGetLastError();
}
hipError_t launch_field_setup(const ChainDev* d_cd, int ci, const double* h, double beta, int64_t N, int precision,
                              hipStream_t s) {
  if (precision == 4) k_field_setup<float><<<nblk(N), 256, 0, s>>>(d_cd, ci, h, beta);
  else k_field_setup<double><<<nblk(N), 256, 0, s>>>(d_cd, ci, h, beta);
  return hipGetLastError();
}
hipError_t launch_field_cg(ChainDev* d_cd, const int* which, int n, double* work, const int64_t* woff,
                           hipStream_t s) {
  if (n > 0) k_field_cg<<<(unsigned)n, 256, 0, s>>>(d_cd, which, work, woff);
  return hipGetLastError();
}
hipError_t launch_measure(const std::vector<Group>& groups, const Tile* d_tiles, const ChainDev* d_cd, hipStream_t s) {
  for (auto& g : groups) {
    hipError_t e = launch_lattice_pass(g.prec, g.ndim, g.cls, PASS_MEASURE, d_cd, d_tiles + g.tile_off,
                                       g.tile_begin.back(), 0, 0, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t setup_partials(ChainDev& c, void* block, hipStream_t s) {
  char* b = (char*)block;
  const uint64_t ng = part_groups(c.n_tiles);
  c.part = (uint64_t*)b;
  b += ((uint64_t)c.n_tiles * NPART * 16 + 255) / 256 * 256;
  c.gsum = (uint64_t*)b;
  b += (ng * NPART * 16 + 255) / 256 * 256;
  c.gcnt = (uint32_t*)b;
  return hipMemsetAsync(c.gcnt, 0, 4 * ng, s);
}
hipError_t launch_zero_state(ChainState* st, hipStream_t s) {
  k_zero_state<<<1, 256, 0, s>>>(st);
  return hipGetLastError();
}
hipError_t launch_export_psi(const ChainDev* d_cd, int ci, double* out, int64_t N, int precision, hipStream_t s) {
  if (precision == 4) k_export_psi<float><<<nblk(N), 256, 0, s>>>(d_cd, ci, out);
  else k_export_psi<double><<<nblk(N), 256, 0, s>>>(d_cd, ci, out);
  return hipGetLastError();
}
hipError_t launch_export_field(const ChainDev* d_cd, int ci, double* out, const void* src, int64_t N, int precision,
                               hipStream_t s) {
  if (precision == 4) k_export<float><<<nblk(N), 256, 0, s>>>(d_cd, ci, out, (const float*)src);
  else k_export<double><<<nblk(N), 256, 0, s>>>(d_cd, ci, out, (const double*)src);
  return hipGetLastError();
}
}  // namespace ihmc
