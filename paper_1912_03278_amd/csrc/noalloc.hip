// Allocation-free force evaluation (ihmc_force_noalloc): the force pass of the
// lattice path (Sec. 3 equations of motion) on caller-owned device arrays, for
// callers that cannot allocate device memory (code under stream capture, tight
// serving loops).  The chain descriptor, tile table and padded field staging
// live in one file-scope device array; each GPU holds its own copy, whose
// address is looked up once per device when a context is created on it.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "device_common.hpp"
#include "lattice_kernels.hpp"
#include "runtime_internal.hpp"

namespace ihmc {

// Scratch of the allocation-free entry point: 32 MiB per GPU, enough for a
// chain of about 3.9M FP32 or 1.9M FP64 sites (two field arrays plus tiles).
constexpr uint64_t kNoallocBytes = 32ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
static void* g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

// Device address of this GPU's scratch array; the current device must be
// `device`.  Looked up once per device.
int noalloc_scratch_init(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return set_error(IHMC_E_UNSUPPORTED, "device index %d too large", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(IHMC_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return IHMC_OK;
}

namespace {
constexpr uint64_t kOffState = 512, kOffTiles = 1024;
static_assert(sizeof(ChainDev) <= kOffState && sizeof(ChainState) <= kOffTiles - kOffState, "scratch header");
inline uint64_t r256(uint64_t b) { return (b + 255ull) & ~255ull; }

struct NoallocLayout {
  uint64_t tiles, psi, p, end;
};
NoallocLayout layout(const ChainDev& c) {
  NoallocLayout l;
  l.tiles = kOffTiles;
  l.psi = l.tiles + r256(sizeof(Tile) * (uint64_t)c.n_tiles);
  l.p = l.psi + r256((uint64_t)c.NP * (uint64_t)c.precision);
  l.end = l.p + r256((uint64_t)c.NP * (uint64_t)c.precision);
  return l;
}

// Descriptor, a fresh state (accepted field in buffer 0, sign +1) and the tile
// table, written into the scratch at `base` (the kernels only ever see it
// through this pointer).  Tiles in the order of the chain sets: x fastest.
__global__ void k_noalloc_setup(ChainDev c, unsigned char* base, uint64_t off_psi, uint64_t off_p, int bx, int by,
                                int bz) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t == 0) {
    c.psi = base + off_psi;
    c.p = base + off_p;
    c.st = (ChainState*)(base + kOffState);
    *(ChainDev*)base = c;
    uint64_t* w = (uint64_t*)(base + kOffState);
    for (int i = 0; i < (int)(sizeof(ChainState) / 8); ++i) w[i] = 0ull;
    c.st->sign = 1;
  }
  if (t < (int64_t)c.n_tiles) {
    const int nx = (c.L0 + bx - 1) / bx, ny = (c.L1 + by - 1) / by;
    Tile tl;
    tl.chain = 0;
    tl.x0 = (int)(t % nx) * bx;
    tl.y0 = (int)((t / nx) % ny) * by;
    tl.z0 = (int)(t / ((int64_t)nx * ny)) * bz;
    ((Tile*)(base + kOffTiles))[t] = tl;
  }
}

// Caller's field (site order) into the padded stored layout; padding zeroed.
template <typename T>
__global__ void k_noalloc_import(const unsigned char* base, const T* __restrict__ src) {
  const ChainDev& c = *(const ChainDev*)base;
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= c.NP) return;
  const int64_t x = k % c.pitch, r = k / c.pitch;
  ((T*)c.psi)[k] = x < c.L0 ? src[x + (int64_t)c.L0 * r] : (T)0;
}

// The force (written to momentum buffer 0 by the force pass) back to site order.
template <typename T>
__global__ void k_noalloc_export(const unsigned char* base, T* __restrict__ dst) {
  const ChainDev& c = *(const ChainDev*)base;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < c.N) dst[i] = ((const T*)c.p)[stored_index(c, i)];
}
}  // namespace

}  // namespace ihmc

using namespace ihmc;

extern "C" int ihmc_force_noalloc(ihmc_ctx* ctx, const ihmc_lattice* lat, int32_t precision, const void* psi,
                                  void* F, void* stream) {
  CTX_OK(ctx);
  if (!lat || !psi || !F) return set_error(IHMC_E_INVAL, "NULL argument");
  if (!ctx->scratch) return set_error(IHMC_E_DEVICE, "no scratch array on this device");
  ihmc_run r;
  std::memset(&r, 0, sizeof r);
  r.n_md = 1;
  r.n_traj = 1;
  r.traj_len = 1.0;
  r.precision = precision;
  int rc = validate(*lat, r, 0);
  if (rc) return rc;
  if (lat->h_len > 1)
    return set_error(IHMC_E_UNSUPPORTED, "the allocation-free force takes h = 0 or a uniform field only");
  ChainDev c;
  describe_chain(*lat, r, BUILD_TILED, ctx->tune.class_for(tile_key(*lat, precision)), c);
  const NoallocLayout l = layout(c);
  if (l.end > kNoallocBytes)
    return set_error(IHMC_E_INVAL, "lattice of %lld sites needs %llu bytes of scratch, the maximum is %llu",
                     (long long)c.N, (unsigned long long)l.end, (unsigned long long)kNoallocBytes);
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  unsigned char* base = (unsigned char*)ctx->scratch;
  const TileShape ts = tile_shape(c.precision, c.ndim, c.tile_cls);
  const unsigned tb = (unsigned)((c.n_tiles + 255) / 256);
  k_noalloc_setup<<<tb, 256, 0, s>>>(c, base, l.psi, l.p, ts.bx, ts.by, ts.bz);
  hipError_t e = hipGetLastError();
  const unsigned nb = (unsigned)((c.NP + 255) / 256), ns = (unsigned)((c.N + 255) / 256);
  if (e == hipSuccess) {
    if (precision == 4) k_noalloc_import<float><<<nb, 256, 0, s>>>(base, (const float*)psi);
    else k_noalloc_import<double><<<nb, 256, 0, s>>>(base, (const double*)psi);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = launch_lattice_pass(c.precision, c.ndim, c.tile_cls, PASS_FORCE, (const ChainDev*)base,
                            (const Tile*)(base + kOffTiles), (int)c.n_tiles, 0, 0, s);
  if (e == hipSuccess) {
    if (precision == 4) k_noalloc_export<float><<<ns, 256, 0, s>>>(base, (float*)F);
    else k_noalloc_export<double><<<ns, 256, 0, s>>>(base, (double*)F);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "allocation-free force");
  return IHMC_OK;
}
