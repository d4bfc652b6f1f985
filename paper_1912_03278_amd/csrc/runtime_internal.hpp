// Host-side runtime objects behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/ihmc.h"
#include "ihmc_internal.hpp"

namespace ihmc {

int set_error(int code, const char* fmt, ...);
int hip_fail(ihmc_ctx* ctx, hipError_t e, const char* where);

// Set-up launchers shared by the lattice and dense runtimes (runtime.hip).
hipError_t launch_init_psi(const ChainDev* d_cd, int ci, const double* psi0, int64_t N, int precision, hipStream_t s,
                           const double* shift = nullptr);
hipError_t launch_scale(double* x, int64_t n, double by, hipStream_t s);  // x /= by
hipError_t launch_zero_state(ChainState* st, hipStream_t s);
// Point c.part / c.gsum / c.gcnt into `block` (partials_bytes(c.n_tiles) bytes)
// and clear the group counters.
hipError_t setup_partials(ChainDev& c, void* block, hipStream_t s);
hipError_t launch_export_psi(const ChainDev* d_cd, int ci, double* out, int64_t N, int precision, hipStream_t s);
hipError_t launch_export_field(const ChainDev* d_cd, int ci, double* out, const void* src, int64_t N, int precision,
                               hipStream_t s);
int result_from_device(ihmc_ctx* ctx, const ChainDev& c, const ChainDev* d_cd, int ci, ihmc_result* out);
// Checkpoint of one chain into a host buffer (buf NULL: size only), and its
// restore into a chain with the same parameters (sets *traj to the
// checkpoint's trajectory index).  `variant` names a path-specific form of the
// force that must also match (0 for the lattice path).  Both wait for stream
// s (null: the context stream) and do their copies on it.
int chain_checkpoint(ihmc_ctx* ctx, const ChainDev& c, uint64_t variant, void* buf, uint64_t* bytes,
                     hipStream_t s = nullptr);
int chain_restore(ihmc_ctx* ctx, const ChainDev& c, uint64_t variant, const void* buf, uint64_t bytes, int* traj,
                  hipStream_t s = nullptr);
// The same checkpoint built from host copies of a finished lattice chain: its
// state, its accepted field in site order with the sign applied, and its
// records; fh = field_hash_host of its h' in site order (0 without a per-site field).
int chain_checkpoint_host(const ChainDev& c, uint64_t fh, const ChainState& st, const double* psi,
                          const TrajRecord* rec, int n_rec, std::vector<char>& out);
// Largest checkpoint of a chain (all cap records).
uint64_t chain_checkpoint_max_bytes(const ChainDev& c);
uint64_t field_hash_host(const double* hp, int64_t n);

// First-fit sub-allocator over one device allocation (256-byte granules).
struct Arena {
  char* base = nullptr;
  uint64_t size = 0;
  uint64_t used = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> bytes
  std::map<uint64_t, uint64_t> live_;  // offset -> bytes
  std::mutex mu;
  void* alloc(uint64_t bytes);
  void release(void* p);
};

enum BuildFlags : int { BUILD_P_GIVEN = 1, BUILD_WRITE_P = 2, BUILD_TILED = 4 };  // TILED: never LDS-resident

// Tile classes of the lattice passes: the built-in rule (lattice_kernels.hip)
// and the per-shape choices of the autotuner (tune.hip), keyed by what the
// cost of a pass depends on.
struct TileKey {
  int32_t prec, ndim, L0, L1, L2, site_field;
  bool operator<(const TileKey& o) const {
    return std::tie(prec, ndim, L0, L1, L2, site_field) < std::tie(o.prec, o.ndim, o.L0, o.L1, o.L2, o.site_field);
  }
};
constexpr int kMaxTileClasses = 4;
struct TuneEntry {
  int32_t cls = 0;
  int32_t source = IHMC_TUNE_RULE;
  double ns_site[kMaxTileClasses];  // middle-pass ns per site of each class (NaN: not measured)
};
struct TuneTable {
  std::mutex mu;
  std::map<TileKey, TuneEntry> m;
  // The table's class for k, else the built-in rule.
  int class_for(const TileKey& k);
};
TileKey tile_key(const ihmc_lattice& l, int precision);
// Launch class of a new chain: RESIDENT_CLASS when the context allows and the
// chain fits one workgroup's LDS (and no diagnostic flag is set), else the
// tuning table's tile class (or the built-in rule's).
int choose_class(ihmc_ctx* ctx, const ihmc_lattice& l, int precision, int flags, int form = 0);
// JSON form of the table; load merges (entries replace equal keys).
int tune_save(TuneTable& t, const char* path);
int tune_load(TuneTable& t, const char* path);

// Chains of equal state precision and dimension share launches.
struct Group {
  int prec = 4, ndim = 2, cls = 0;
  bool pair = false;            // middle steps two per launch (PASS_PAIR)
  std::vector<int> order;       // chain indices, sorted by pass count (descending)
  std::vector<int> n_pass;      // pass count per position in `order`
  std::vector<int> tile_begin;  // first tile of each position, relative to tile_off; size+1
  int tile_off = 0;
  int max_pass = 0;
};

// Chain descriptors, launch plans and rounds shared by the resident chain sets
// and the serving loop (runtime.hip).
int validate(const ihmc_lattice& l, const ihmc_run& r, int idx);
int64_t lattice_sites(const ihmc_lattice& l);
// Descriptor of one chain whose passes use tile class `cls` (no device memory).
void describe_chain(const ihmc_lattice& l, const ihmc_run& r, int flags, int cls, ChainDev& c);
uint32_t chain_tile_count(const ChainDev& c);
// fuse_steps: 2D tiled groups run their middle steps two per launch.
void plan_groups(const std::vector<ChainDev>& cd, const std::vector<int>& members, std::vector<Group>& groups,
                 std::vector<Tile>& tiles, bool fuse_steps);
size_t round_events(const std::vector<Group>& groups);
// Events the round of a plan actually takes (a dry run of the enqueue that
// makes no HIP call); never more than round_events(groups).
size_t round_events_used(const std::vector<Group>& groups);
// One trajectory of every chain of the plan: FIRST over all tiles of a group,
// then the middle steps per pass index, then one LAST launch that runs every
// chain's own last pass; each group on a side stream of its own.
hipError_t enqueue_round_plan(const std::vector<Group>& groups, const Tile* d_tiles, const ChainDev* d_cd,
                              const std::vector<hipStream_t>& side, const std::vector<hipEvent_t>& events,
                              hipStream_t s);
// Per-site field of chain ci into its stored layout (h: device, logical order).
hipError_t launch_field_setup(const ChainDev* d_cd, int ci, const double* h, double beta, int64_t N, int precision,
                              hipStream_t s);
// h'^T Kt^-1 h' and 1^T Kt^-1 h' of the chains `which` (device int array, n
// entries) by CG, one block per chain; work: 4 N doubles per chain at woff.
hipError_t launch_field_cg(ChainDev* d_cd, const int* which, int n, double* work, const int64_t* woff,
                           hipStream_t s);
hipError_t launch_measure(const std::vector<Group>& groups, const Tile* d_tiles, const ChainDev* d_cd, hipStream_t s);
hipError_t launch_resident_group(const Group& g, const ChainDev* d_cd, const Tile* t, int n, int n_traj,
                                 int per_cu, hipStream_t s);

struct Chains {
  ihmc_ctx* ctx = nullptr;
  int n = 0;
  std::vector<ChainDev> cd;  // host copies
  ChainDev* d_cd = nullptr;
  Tile* d_tiles = nullptr;
  std::vector<Group> groups;
  std::vector<void*> allocs;
  std::vector<hipStream_t> side;   // one per launch group
  std::vector<hipEvent_t> events;  // fork/join points of one round
  int enqueued = 0;
  std::vector<int> base;  // per chain: trajectory index at enqueued = 0 (non-zero after a restore)
  // A shifted-form chain with a per-site field runs as a paper-form chain in
  // coordinates translated by delta = Kt^-1 h'/sqrt(J'): HMC with unit mass
  // commutes with translations, and the two actions differ by the constant
  // h'.Kt^-1 h'/(2J').  Per chain: delta (logical layout) and that offset, or
  // an empty vector and 0.
  std::vector<std::vector<double>> delta;
  std::vector<double> s_offset;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;

  void* dalloc(uint64_t bytes);
  int build(int32_t n, const ihmc_lattice* lats, const ihmc_run* runs, int flags);
  hipError_t enqueue_round(hipStream_t s);
  int advance(int32_t n_traj);
  int checkpoint(int32_t i, void* buf, uint64_t* bytes);
  int restore(int32_t i, const void* buf, uint64_t bytes);
  int result(int32_t i, ihmc_result* out);
  ~Chains();
};

}  // namespace ihmc

#define HIPCHK(expr, what)                                \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) return hip_fail(ctx, _e, what); \
  } while (0)

#define CTX_OK(c)                                                                             \
  do {                                                                                        \
    if (!(c)) return set_error(IHMC_E_INVAL, "ctx is NULL");                                  \
    if ((c)->dead) return set_error(IHMC_E_DEVICE, "context is unusable after a device error"); \
    hipSetDevice((c)->device);                                                                \
  } while (0)

struct ihmc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  ihmc::Arena arena;
  ihmc_alloc_fn af = nullptr;
  ihmc_free_fn ff = nullptr;
  void* user = nullptr;
  bool dead = false;
  ihmc::TuneTable tune;
  int64_t resident_sites = -1;  // chains up to this many sites run LDS-resident (-1: as many as fit, 0: none)
  int32_t fuse_steps = 1;       // 2D tiled chains run two middle steps per launch
  void* scratch = nullptr;      // this device's scratch of the allocation-free entry point
};

namespace ihmc {
// Device address of the allocation-free entry point's scratch array on
// `device` (the current device), looked up once per device (noalloc.hip).
int noalloc_scratch_init(int device, void** out);
}  // namespace ihmc
