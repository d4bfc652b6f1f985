// Serving loop: continuous batching of HMC requests.
//
// Requests (one lattice chain each) are submitted asynchronously.  A scheduler
// thread owns the device side: before every round it admits queued requests,
// in arrival order, while their device footprint fits the server's HBM budget
// and a chain slot is free, sets them up (initial field, S(psi0)), then advances
// every resident chain by one trajectory with the fused lattice passes, and
// retires the chains that reached their trajectory count: their series, state
// and final field are copied to host memory, their device memory and slot are
// released, and the next queued requests take their place.  Chain state stays
// on the device between rounds.  A chain's arithmetic depends only on its own
// parameters (fixed-point sums, per-site work independent of the tile and of
// the other chains in a launch), so a served result is bit-identical to the
// same request run alone.  A round is enqueued while the previous one still
// runs (the host's per-request trajectory counts advance at enqueue); the
// set-up of admitted requests, retirement and checkpoints wait for the rounds
// in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "lattice_kernels.hpp"
#include "runtime_internal.hpp"

using namespace ihmc;

namespace ihmc {

enum ReqState : int32_t { REQ_QUEUED = 0, REQ_RUNNING = 1, REQ_DONE = 2, REQ_CANCELLED = 3, REQ_FAILED = 4 };

struct Request {
  uint64_t ticket = 0;
  int32_t state = REQ_QUEUED;
  ihmc_lattice lat{};
  ihmc_run run{};
  std::vector<double> h, psi0;
  std::vector<uint8_t> replay;
  uint64_t need = 0;  // device bytes while resident
  int cls = 0;        // tile class, fixed at submission
  int slot = -1;
  ChainDev cd{};
  std::vector<void*> dev;  // arena blocks
  int rounds = 0;
  bool cancel = false;
  std::vector<TrajRecord> rec;
  ChainState st{};
  std::vector<double> psi;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int err_code = 0;
  std::string error;
  std::vector<char> resume;  // chain checkpoint to continue from (restored requests)
  bool ckpt_wanted = false;  // a checkpoint is asked for at the next round boundary
  bool ckpt_ready = false;
  std::vector<char> ckpt;    // the chain checkpoint taken by the scheduler
  // A shifted-form request with a per-site field runs in coordinates
  // translated by delta = Kt^-1 h'/sqrt(J') (as a chain set does): delta in the
  // logical layout and the action offset h'.Kt^-1 h'/(2J'), applied at fetch.
  std::vector<double> delta;
  double s_off = 0.0;
  const double* dshift = nullptr;  // device delta during the set-up
};

static inline uint64_t r256(uint64_t b) { return (b + 255ull) & ~255ull; }

// Device bytes a request holds while resident (state, records, field arrays,
// and its share of the tile table), plus its set-up staging.
static uint64_t request_bytes(const ihmc_lattice& l, const ihmc_run& r, int cls) {
  const int64_t N = lattice_sites(l);
  const int64_t pitch = (l.L[0] + 3) & ~3;
  const int64_t NP = pitch * (N / l.L[0]);
  const uint64_t pb = (uint64_t)r.precision;
  uint64_t b = r256((uint64_t)LAT_BUFFERS * NP * pb) + r256((uint64_t)LAT_P_BUFFERS * NP * pb) +
               r256(sizeof(TrajRecord) * (uint64_t)std::max(1, r.n_traj)) + r256(sizeof(ChainState)) +
               r256(8 * (uint64_t)N);
  if (r.replay_accept) b += r256((uint64_t)r.n_traj);
  if (l.h_len == N && N > 1) b += r256(8 * NP) + r256(NP * pb) + r256(8 * 4 * (uint64_t)N) + r256(8 * (uint64_t)N);
  ChainDev c;
  describe_chain(l, r, 0, cls, c);
  b += r256(sizeof(Tile) * (uint64_t)c.n_tiles) + partials_bytes(c.n_tiles);
  return b;
}

// Checkpoint of a served request: the request itself (lattice, run
// parameters, field, given initial field, replayed decisions) and, once it has
// run, its chain checkpoint (chain_checkpoint's format).  A request restored
// from it continues where the checkpoint was taken, bit for bit.
constexpr char kSrvMagic[8] = {'I', 'H', 'M', 'C', 'S', 'R', 'V', 'C'};
constexpr uint32_t kSrvVersion = 2;  // 2: the run's form
struct SrvHeader {
  char magic[8];
  uint32_t version, header_bytes;
  int32_t ndim, L[3];
  double J, beta, C;
  int64_t h_len;
  int32_t n_md, n_traj;
  double traj_len;
  int32_t integrator, flip_every, precision, n_therm;
  uint64_t seed, chain_id;
  int64_t psi0_len, replay_len;
  uint64_t chain_bytes;
  int32_t form, pad;
};

static uint64_t served_prefix_bytes(const Request* r) {
  return sizeof(SrvHeader) + 8 * (uint64_t)r->h.size() + 8 * (uint64_t)r->psi0.size() + (uint64_t)r->replay.size();
}

static void served_write(const Request* r, const std::vector<char>& chain, std::vector<char>& out) {
  SrvHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, kSrvMagic, 8);
  h.version = kSrvVersion;
  h.header_bytes = sizeof h;
  h.ndim = r->lat.ndim;
  for (int i = 0; i < 3; ++i) h.L[i] = r->lat.L[i];
  h.J = r->lat.J;
  h.beta = r->lat.beta;
  h.C = r->lat.C;
  h.h_len = (int64_t)r->h.size();
  h.n_md = r->run.n_md;
  h.n_traj = r->run.n_traj;
  h.traj_len = r->run.traj_len;
  h.integrator = r->run.integrator;
  h.flip_every = r->run.flip_every;
  h.precision = r->run.precision;
  h.n_therm = r->run.n_therm;
  h.form = r->run.form;
  h.seed = r->run.seed;
  h.chain_id = r->run.chain_id;
  h.psi0_len = (int64_t)r->psi0.size();
  h.replay_len = (int64_t)r->replay.size();
  h.chain_bytes = chain.size();
  out.resize(served_prefix_bytes(r) + chain.size());
  char* o = out.data();
  std::memcpy(o, &h, sizeof h);
  o += sizeof h;
  if (!r->h.empty()) std::memcpy(o, r->h.data(), 8 * r->h.size());
  o += 8 * r->h.size();
  if (!r->psi0.empty()) std::memcpy(o, r->psi0.data(), 8 * r->psi0.size());
  o += 8 * r->psi0.size();
  if (!r->replay.empty()) std::memcpy(o, r->replay.data(), r->replay.size());
  o += r->replay.size();
  if (!chain.empty()) std::memcpy(o, chain.data(), chain.size());
}

}  // namespace ihmc

struct ihmc_server {
  ihmc_ctx* ctx = nullptr;
  uint64_t budget = 0;
  int max_active = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread th;
  bool stop = false;
  std::deque<Request*> queue;
  std::vector<Request*> active;
  std::map<uint64_t, Request*> reqs;
  uint64_t next_ticket = 1, used = 0;
  // device side (scheduler thread only)
  hipStream_t s = nullptr;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> events;
  ChainDev* d_cd = nullptr;
  std::vector<ChainDev> cd_host;  // slot table
  std::vector<int> free_slots;
  Tile* d_tiles = nullptr;
  Tile* h_tiles = nullptr;  // pinned staging of the tile table (set-up of admitted chains)
  size_t tile_cap = 0;
  // the rounds' tile tables, two of each: a round is enqueued while the one
  // before it still runs, so its table goes to the other buffer; copy_ev[b]
  // marks the upload from rh_tiles[b], which the host waits for before it
  // writes that staging buffer again
  Tile* rd_tiles[2] = {nullptr, nullptr};
  Tile* rh_tiles[2] = {nullptr, nullptr};
  hipEvent_t copy_ev[2] = {nullptr, nullptr};
  bool copy_pending[2] = {false, false};
  size_t rtile_cap = 0;
  int round_buf = 0;
  double* d_export = nullptr;
  int64_t export_cap = 0;
  // statistics
  std::chrono::steady_clock::time_point t0;
  int64_t rounds = 0, completed = 0;
  double busy_s = 0.0, site_steps = 0.0;
  int max_seen = 0;
  bool dead = false;
  std::string dead_msg;

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
  void loop();
  bool admit_setup(std::vector<Request*>& fresh);
  bool run_round();
  void retire(Request* r, int32_t final_state);
  void fail_all(const char* what, hipError_t e);
  bool ensure_tiles(size_t n);
  bool ensure_round_tiles(size_t n);
  bool ensure_streams(size_t n_groups, size_t n_events);
  void take_checkpoints();
  void resume_requests(std::vector<Request*>& ok);
};

// Checkpoints asked for since the last round, taken while the device is idle
// between rounds.  Scheduler thread.
void ihmc_server::take_checkpoints() {
  std::vector<Request*> want;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (Request* r : active)
      if (r->ckpt_wanted && !r->ckpt_ready) want.push_back(r);
  }
  for (Request* r : want) {
    const ChainDev& c = cd_host[r->slot];
    uint64_t n = 0;
    std::vector<char> blob;
    int rc = chain_checkpoint(ctx, c, 0, nullptr, &n, s);
    if (rc == IHMC_OK) {
      blob.resize(n);
      rc = chain_checkpoint(ctx, c, 0, blob.data(), &n, s);
      blob.resize(n);
    }
    std::lock_guard<std::mutex> lk(mu);
    r->ckpt_wanted = false;
    if (rc == IHMC_OK) {
      r->ckpt.swap(blob);
      r->ckpt_ready = true;
    } else {
      r->ckpt.clear();
      r->ckpt_ready = true;  // empty: the checkpoint failed
    }
    cv_done.notify_all();
  }
}

// Restored requests: replace the freshly set-up state of each admitted chain
// with its checkpoint.  Scheduler thread, device idle.
void ihmc_server::resume_requests(std::vector<Request*>& ok) {
  for (auto it = ok.begin(); it != ok.end();) {
    Request* r = *it;
    if (r->resume.empty()) {
      ++it;
      continue;
    }
    int traj = 0;
    const int rc = chain_restore(ctx, cd_host[r->slot], 0, r->resume.data(), r->resume.size(), &traj, s);
    if (rc == IHMC_OK) {
      std::lock_guard<std::mutex> lk(mu);
      r->rounds = traj;
      r->resume.clear();
      ++it;
      continue;
    }
    for (void* p : r->dev) ctx->arena.release(p);
    r->dev.clear();
    std::lock_guard<std::mutex> lk(mu);
    used -= r->need;
    free_slots.push_back(r->slot);
    r->state = REQ_FAILED;
    r->err_code = rc;
    r->error = std::string("restore: ") + ihmc_last_error();
    r->t_done = now();
    cv_done.notify_all();
    it = ok.erase(it);
  }
}

void ihmc_server::fail_all(const char* what, hipError_t e) {
  std::lock_guard<std::mutex> lk(mu);
  dead = true;
  dead_msg = std::string(what) + ": " + hipGetErrorString(e);
  ctx->dead = true;
  for (Request* r : active) {
    r->state = REQ_FAILED;
    r->err_code = IHMC_E_DEVICE;
    r->error = dead_msg;
  }
  active.clear();
  for (Request* r : queue) {
    r->state = REQ_FAILED;
    r->err_code = IHMC_E_DEVICE;
    r->error = dead_msg;
  }
  queue.clear();
  cv_done.notify_all();
}

bool ihmc_server::ensure_tiles(size_t n) {
  if (n <= tile_cap) return true;
  const size_t cap = std::max<size_t>(n, 2 * tile_cap);
  if (d_tiles) ctx->arena.release(d_tiles);
  if (h_tiles) hipHostFree(h_tiles);
  d_tiles = nullptr;
  h_tiles = nullptr;
  tile_cap = 0;
  d_tiles = (Tile*)ctx->arena.alloc(sizeof(Tile) * cap);
  if (!d_tiles) return false;
  if (hipHostMalloc((void**)&h_tiles, sizeof(Tile) * cap, 0) != hipSuccess) {
    h_tiles = nullptr;
    ctx->arena.release(d_tiles);
    d_tiles = nullptr;
    return false;
  }
  tile_cap = cap;
  return true;
}

// Both round tile tables with room for n tiles.  Growing them waits for the
// rounds in flight, which read the old ones.
bool ihmc_server::ensure_round_tiles(size_t n) {
  if (n <= rtile_cap) return true;
  if (hipStreamSynchronize(s) != hipSuccess) return false;
  const size_t cap = std::max<size_t>(n, 2 * rtile_cap);
  for (int b = 0; b < 2; ++b) {
    if (rd_tiles[b]) ctx->arena.release(rd_tiles[b]);
    if (rh_tiles[b]) hipHostFree(rh_tiles[b]);
    rd_tiles[b] = nullptr;
    rh_tiles[b] = nullptr;
    copy_pending[b] = false;
  }
  rtile_cap = 0;
  for (int b = 0; b < 2; ++b) {
    if (!copy_ev[b] && hipEventCreateWithFlags(&copy_ev[b], hipEventDisableTiming) != hipSuccess) return false;
    rd_tiles[b] = (Tile*)ctx->arena.alloc(sizeof(Tile) * cap);
    if (!rd_tiles[b]) return false;
    if (hipHostMalloc((void**)&rh_tiles[b], sizeof(Tile) * cap, 0) != hipSuccess) {
      rh_tiles[b] = nullptr;
      return false;
    }
  }
  rtile_cap = cap;
  return true;
}

bool ihmc_server::ensure_streams(size_t n_groups, size_t n_events) {
  while (side.size() < n_groups) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return false;
    side.push_back(st);
  }
  while (events.size() < n_events) {
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return false;
    events.push_back(ev);
  }
  return true;
}

// Copy a finished (or cancelled) chain's results to host memory and release
// its device memory and slot.  Scheduler thread; the stream is idle.
void ihmc_server::retire(Request* r, int32_t final_state) {
  const ChainDev& c = cd_host[r->slot];
  hipError_t e = hipMemcpyAsync(&r->st, c.st, sizeof(ChainState), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const int done = std::min(r->st.traj, c.cap);
  if (e == hipSuccess && done > 0) {
    r->rec.resize(done);
    e = hipMemcpyAsync(r->rec.data(), c.rec, sizeof(TrajRecord) * done, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (e == hipSuccess) {
    if (c.N > export_cap) {
      if (d_export) ctx->arena.release(d_export);
      d_export = (double*)ctx->arena.alloc(8 * (uint64_t)c.N);
      export_cap = d_export ? c.N : 0;
    }
    if (d_export) {
      r->psi.resize(c.N);
      e = launch_export_psi(d_cd, r->slot, d_export, c.N, c.precision, s);
      if (e == hipSuccess) e = hipMemcpyAsync(r->psi.data(), d_export, 8 * c.N, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
  }
  for (void* p : r->dev) ctx->arena.release(p);
  r->dev.clear();
  std::lock_guard<std::mutex> lk(mu);
  free_slots.push_back(r->slot);
  used -= r->need;
  r->t_done = now();
  if (e != hipSuccess) {
    r->state = REQ_FAILED;
    r->err_code = IHMC_E_DEVICE;
    r->error = std::string("result copy: ") + hipGetErrorString(e);
  } else {
    r->state = final_state;
    if (final_state == REQ_DONE) ++completed;
  }
  cv_done.notify_all();
}

// Device set-up of newly admitted requests: memory, descriptor upload, initial
// field, per-site field constants, and the measurement of S(psi0).
bool ihmc_server::admit_setup(std::vector<Request*>& fresh) {
  std::vector<void*> temps;
  auto tmp = [&](uint64_t b) {
    void* p = ctx->arena.alloc(b);
    if (p) temps.push_back(p);
    return p;
  };
  std::vector<Request*> ok;
  std::vector<int> cg_slots;
  std::vector<int64_t> cg_off;
  int64_t cg_total = 0;
  // the set-up runs with the device idle: the round in flight finishes first
  hipError_t e = hipStreamSynchronize(s);
  for (Request* r : fresh) {
    if (e != hipSuccess) break;
    ChainDev& c = r->cd;
    describe_chain(r->lat, r->run, 0, r->cls, c);
    const uint64_t pb = (uint64_t)c.precision;
    auto dal = [&](uint64_t b) {
      void* p = ctx->arena.alloc(b);
      if (p) r->dev.push_back(p);
      return p;
    };
    c.psi = dal((uint64_t)LAT_BUFFERS * c.NP * pb);
    c.p = dal((uint64_t)LAT_P_BUFFERS * c.NP * pb);
    c.rec = (TrajRecord*)dal(sizeof(TrajRecord) * (uint64_t)std::max(1, r->run.n_traj));
    c.st = (ChainState*)dal(sizeof(ChainState));
    void* pblk = dal(partials_bytes(c.n_tiles));
    bool good = c.psi && c.p && c.rec && c.st && pblk;
    if (good) e = setup_partials(c, pblk, s);
    if (good && !r->replay.empty()) {
      uint8_t* d = (uint8_t*)dal(r->replay.size());
      good = d != nullptr;
      if (good) e = hipMemcpyAsync(d, r->replay.data(), r->replay.size(), hipMemcpyHostToDevice, s);
      c.replay = d;
    }
    if (good && c.h_kind == 2) {
      c.hp = (double*)dal(8 * (uint64_t)c.NP);
      c.b = dal((uint64_t)c.NP * pb);
      good = c.hp && c.b;
    }
    if (!good || e != hipSuccess) {
      for (void* p : r->dev) ctx->arena.release(p);
      r->dev.clear();
      std::lock_guard<std::mutex> lk(mu);
      used -= r->need;
      free_slots.push_back(r->slot);
      r->state = REQ_FAILED;
      r->err_code = e != hipSuccess ? IHMC_E_DEVICE : IHMC_E_NOMEM;
      r->error = e != hipSuccess ? "replay upload failed" : "device arena exhausted at admission";
      r->t_done = now();
      cv_done.notify_all();
      if (e != hipSuccess) break;
      continue;
    }
    cd_host[r->slot] = c;
    e = hipMemcpyAsync(d_cd + r->slot, &cd_host[r->slot], sizeof(ChainDev), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_zero_state(c.st, s);
    if (e == hipSuccess && c.h_kind == 2) {
      double* t = (double*)tmp(8 * (uint64_t)c.N);
      if (!t) e = hipErrorOutOfMemory;
      if (e == hipSuccess) e = hipMemcpyAsync(t, r->h.data(), 8 * c.N, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = launch_field_setup(d_cd, r->slot, t, r->lat.beta, c.N, c.precision, s);
      cg_slots.push_back(r->slot);
      cg_off.push_back(cg_total);
      cg_total += 4 * c.N;
    }
    const bool translated = r->run.form == FORM_SHIFTED && c.h_kind == 2;
    if (e == hipSuccess) {
      const double* src = nullptr;
      if (!r->psi0.empty()) {
        double* t = (double*)tmp(8 * (uint64_t)c.N);
        if (!t) e = hipErrorOutOfMemory;
        if (e == hipSuccess) e = hipMemcpyAsync(t, r->psi0.data(), 8 * c.N, hipMemcpyHostToDevice, s);
        src = t;
      }
      // a translated request's field starts after the CG below, with delta added
      if (e == hipSuccess && !translated) e = launch_init_psi(d_cd, r->slot, src, c.N, c.precision, s);
      if (translated) r->dshift = src;  // the staged psi0 (or null), for the later start
    }
    if (e != hipSuccess) break;
    ok.push_back(r);
  }
  if (e == hipSuccess && !cg_slots.empty()) {
    double* work = (double*)tmp(8 * (uint64_t)cg_total);
    int* which = (int*)tmp(sizeof(int) * cg_slots.size());
    int64_t* woff = (int64_t*)tmp(sizeof(int64_t) * cg_off.size());
    if (!work || !which || !woff) e = hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipMemcpyAsync(which, cg_slots.data(), sizeof(int) * cg_slots.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(woff, cg_off.data(), sizeof(int64_t) * cg_off.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_field_cg(d_cd, which, (int)cg_slots.size(), work, woff, s);
    // translated requests: delta = x / sqrt(J') (x = Kt^-1 h' of the CG), then
    // the starting field psi0 + delta, as a chain set starts it
    for (Request* r : ok) {
      if (e != hipSuccess) break;
      if (!(r->run.form == FORM_SHIFTED && r->cd.h_kind == 2)) continue;
      size_t j = 0;
      while (j < cg_slots.size() && cg_slots[j] != r->slot) ++j;
      double* x = work + cg_off[j];
      e = launch_scale(x, r->cd.N, r->cd.sqJ, s);
      if (e == hipSuccess) e = launch_init_psi(d_cd, r->slot, r->dshift, r->cd.N, r->cd.precision, s, x);
      r->dshift = x;
    }
  }
  if (e == hipSuccess && !ok.empty()) {
    std::vector<int> slots;
    for (Request* r : ok) slots.push_back(r->slot);
    std::vector<Group> g;
    std::vector<Tile> tiles;
    plan_groups(cd_host, slots, g, tiles, ctx->fuse_steps != 0);
    if (!ensure_tiles(tiles.size())) {
      e = hipErrorOutOfMemory;
    } else {
      std::memcpy(h_tiles, tiles.data(), sizeof(Tile) * tiles.size());
      e = hipMemcpyAsync(d_tiles, h_tiles, sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = launch_measure(g, d_tiles, d_cd, s);
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  for (Request* r : ok) {  // translated requests: delta and the action offset to the host
    if (e != hipSuccess) break;
    if (!(r->run.form == FORM_SHIFTED && r->cd.h_kind == 2)) continue;
    r->delta.resize((size_t)r->cd.N);
    e = hipMemcpy(r->delta.data(), r->dshift, 8 * (uint64_t)r->cd.N, hipMemcpyDeviceToHost);
    double ce = 0.0;
    if (e == hipSuccess) e = hipMemcpy(&ce, &d_cd[r->slot].c_e, sizeof ce, hipMemcpyDeviceToHost);
    r->s_off = ce / (2.0 * r->cd.Jp);
    r->dshift = nullptr;
  }
  for (void* p : temps) ctx->arena.release(p);
  if (e == hipSuccess) resume_requests(ok);
  if (e != hipSuccess) {
    {
      // requests of this batch are in neither the queue nor the active set yet
      std::lock_guard<std::mutex> lk(mu);
      for (Request* r : fresh)
        if (r->state == REQ_QUEUED) {
          for (void* p : r->dev) ctx->arena.release(p);
          r->dev.clear();
          r->state = REQ_FAILED;
          r->err_code = IHMC_E_DEVICE;
          r->error = "request set-up failed";
        }
    }
    fail_all("request set-up", e);
    return false;
  }
  std::lock_guard<std::mutex> lk(mu);
  for (Request* r : ok) {
    r->state = REQ_RUNNING;
    active.push_back(r);
  }
  max_seen = std::max(max_seen, (int)active.size());
  return true;
}

// One trajectory of every resident chain that has trajectories left.
bool ihmc_server::run_round() {
  std::vector<int> slots;
  double work = 0.0;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (Request* r : active)
      if (!r->cancel && r->rounds < r->run.n_traj) {
        slots.push_back(r->slot);
        work += (double)r->cd.N * r->run.n_md;
      }
  }
  if (slots.empty()) return true;
  std::vector<Group> g;
  std::vector<Tile> tiles;
  plan_groups(cd_host, slots, g, tiles, ctx->fuse_steps != 0);
  // The round is enqueued without waiting for it: the host plans and submits
  // the next round while this one runs (every request advances by exactly one
  // trajectory per round, so the host's counts do not need the device).  Only
  // retirement, admission and checkpoints wait for the rounds in flight.
  const int b = round_buf;
  round_buf ^= 1;
  hipError_t e = hipSuccess;
  if (!ensure_round_tiles(tiles.size()) || !ensure_streams(g.size(), round_events(g))) e = hipErrorOutOfMemory;
  if (e == hipSuccess && copy_pending[b]) {
    e = hipEventSynchronize(copy_ev[b]);  // the upload two rounds back has read rh_tiles[b]
    copy_pending[b] = false;
  }
  if (e == hipSuccess) {
    std::memcpy(rh_tiles[b], tiles.data(), sizeof(Tile) * tiles.size());
    e = hipMemcpyAsync(rd_tiles[b], rh_tiles[b], sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess) e = hipEventRecord(copy_ev[b], s);
  if (e == hipSuccess) copy_pending[b] = true;
  if (e == hipSuccess) e = enqueue_round_plan(g, rd_tiles[b], d_cd, side, events, s);
  if (e != hipSuccess) {
    fail_all("round", e);
    return false;
  }
  std::lock_guard<std::mutex> lk(mu);
  ++rounds;
  site_steps += work;
  for (Request* r : active)
    if (!r->cancel && r->rounds < r->run.n_traj) ++r->rounds;
  return true;
}

void ihmc_server::loop() {
  hipSetDevice(ctx->device);
  for (;;) {
    const auto t_iter = std::chrono::steady_clock::now();
    std::vector<Request*> fresh, finished;
    bool quit = false;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (dead) return;
      if (stop) {
        for (Request* r : active) r->cancel = true;
        quit = true;
      }
      for (Request* r : active)
        if (r->cancel || r->rounds >= r->run.n_traj) finished.push_back(r);
    }
    take_checkpoints();
    for (Request* r : finished) {
      retire(r, r->cancel ? REQ_CANCELLED : REQ_DONE);
      std::lock_guard<std::mutex> lk(mu);
      active.erase(std::find(active.begin(), active.end(), r));
    }
    if (quit) return;
    {
      std::unique_lock<std::mutex> lk(mu);
      while (!queue.empty() && !free_slots.empty()) {
        Request* r = queue.front();
        if (used + r->need > budget && !(active.empty() && fresh.empty())) break;
        queue.pop_front();
        r->slot = free_slots.back();
        free_slots.pop_back();
        used += r->need;
        r->t_admit = now();
        fresh.push_back(r);
      }
      if (active.empty() && fresh.empty()) {
        cv_work.wait(lk, [&] { return stop || !queue.empty(); });
        continue;
      }
    }
    if (!fresh.empty() && !admit_setup(fresh)) return;
    if (!run_round()) return;
    // busy time: the iterations that had resident chains (set-up, retirement and
    // the waits for rounds in flight included)
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_iter).count();
    std::lock_guard<std::mutex> lk(mu);
    busy_s += dt;
  }
}

// ============================================================ C ABI: serving ===

extern "C" int ihmc_server_create(ihmc_ctx* ctx, uint64_t budget_bytes, int32_t max_active, ihmc_server** out) {
  CTX_OK(ctx);
  if (!out) return set_error(IHMC_E_INVAL, "out is NULL");
  *out = nullptr;
  if (max_active <= 0) max_active = 1024;
  if (budget_bytes == 0 || budget_bytes > ctx->arena.size) budget_bytes = ctx->arena.size / 2;
  ihmc_server* sv = new (std::nothrow) ihmc_server();
  if (!sv) return set_error(IHMC_E_NOMEM, "host allocation failed");
  sv->ctx = ctx;
  sv->budget = budget_bytes;
  sv->max_active = max_active;
  sv->t0 = std::chrono::steady_clock::now();
  sv->cd_host.resize(max_active);
  for (int i = max_active - 1; i >= 0; --i) sv->free_slots.push_back(i);
  sv->d_cd = (ChainDev*)ctx->arena.alloc(sizeof(ChainDev) * (uint64_t)max_active);
  hipError_t e = sv->d_cd ? hipStreamCreateWithFlags(&sv->s, hipStreamNonBlocking) : hipErrorOutOfMemory;
  if (e != hipSuccess) {
    if (sv->d_cd) ctx->arena.release(sv->d_cd);
    delete sv;
    return e == hipErrorOutOfMemory ? set_error(IHMC_E_NOMEM, "arena exhausted (slot table)")
                                    : hip_fail(ctx, e, "server stream");
  }
  sv->th = std::thread([sv] { sv->loop(); });
  *out = sv;
  return IHMC_OK;
}

extern "C" int ihmc_server_destroy(ihmc_server* sv) {
  if (!sv) return IHMC_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    for (Request* r : sv->queue) r->state = REQ_CANCELLED;
    sv->queue.clear();
  }
  sv->cv_work.notify_all();
  if (sv->th.joinable()) sv->th.join();
  hipSetDevice(sv->ctx->device);
  if (sv->s) hipStreamSynchronize(sv->s);
  for (Request* r : sv->active)
    for (void* p : r->dev) sv->ctx->arena.release(p);
  for (auto& kv : sv->reqs) delete kv.second;
  for (hipEvent_t ev : sv->events) hipEventDestroy(ev);
  for (hipStream_t st : sv->side) hipStreamDestroy(st);
  if (sv->s) hipStreamDestroy(sv->s);
  if (sv->d_tiles) sv->ctx->arena.release(sv->d_tiles);
  if (sv->h_tiles) hipHostFree(sv->h_tiles);
  for (int b = 0; b < 2; ++b) {
    if (sv->rd_tiles[b]) sv->ctx->arena.release(sv->rd_tiles[b]);
    if (sv->rh_tiles[b]) hipHostFree(sv->rh_tiles[b]);
    if (sv->copy_ev[b]) hipEventDestroy(sv->copy_ev[b]);
  }
  if (sv->d_export) sv->ctx->arena.release(sv->d_export);
  if (sv->d_cd) sv->ctx->arena.release(sv->d_cd);
  delete sv;
  return IHMC_OK;
}

// Queue a request whose host copies are filled in (lat.h, psi0, replay point
// into the request's own vectors).  Thread-safe.
static int queue_request(ihmc_server* sv, Request* r, uint64_t* ticket) {
  r->lat.h = r->h.empty() ? nullptr : r->h.data();
  r->run.psi0 = nullptr;
  r->run.replay_accept = r->replay.empty() ? nullptr : r->replay.data();
  r->cls = choose_class(sv->ctx, r->lat, r->run.precision, 0);
  r->need = request_bytes(r->lat, r->run, r->cls);
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->dead) {
    delete r;
    return set_error(IHMC_E_DEVICE, "server stopped after a device error: %s", sv->dead_msg.c_str());
  }
  if (sv->stop) {
    delete r;
    return set_error(IHMC_E_CANCELLED, "server is shutting down");
  }
  if (r->need > sv->budget) {
    const unsigned long long need = r->need, budget = sv->budget;
    delete r;
    return set_error(IHMC_E_NOMEM, "request needs %llu device bytes, the server budget is %llu", need, budget);
  }
  if (sv->queue.size() >= (size_t)1 << 20) {
    delete r;
    return set_error(IHMC_E_AGAIN, "serving queue full");
  }
  r->ticket = sv->next_ticket++;
  r->t_submit = sv->now();
  sv->reqs[r->ticket] = r;
  sv->queue.push_back(r);
  *ticket = r->ticket;
  sv->cv_work.notify_one();
  return IHMC_OK;
}

extern "C" int ihmc_submit(ihmc_server* sv, const ihmc_lattice* lat, const ihmc_run* run, uint64_t* ticket) {
  if (!sv || !lat || !run || !ticket) return set_error(IHMC_E_INVAL, "NULL argument");
  int rc = validate(*lat, *run, 0);
  if (rc) return rc;
  if (run->form == FORM_PHI) return set_error(IHMC_E_UNSUPPORTED, "the server runs psi-form or shifted-form chains");
  Request* r = new (std::nothrow) Request();
  if (!r) return set_error(IHMC_E_NOMEM, "host allocation failed");
  r->lat = *lat;
  r->run = *run;
  const int64_t N = lattice_sites(*lat);
  if (lat->h_len > 0) r->h.assign(lat->h, lat->h + lat->h_len);
  if (run->psi0) r->psi0.assign(run->psi0, run->psi0 + N);
  if (run->replay_accept && run->n_traj > 0) r->replay.assign(run->replay_accept, run->replay_accept + run->n_traj);
  return queue_request(sv, r, ticket);
}

extern "C" int ihmc_checkpoint(ihmc_server* sv, uint64_t ticket, void* buf, uint64_t* bytes) {
  if (!sv || !bytes) return set_error(IHMC_E_INVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return set_error(IHMC_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second;
  if (r->state == REQ_FAILED) return set_error(IHMC_E_INVAL, "request %llu failed: %s", (unsigned long long)ticket,
                                               r->error.c_str());
  ChainDev c;
  describe_chain(r->lat, r->run, 0, r->cls, c);
  const uint64_t max_bytes = served_prefix_bytes(r) + chain_checkpoint_max_bytes(c);
  if (!buf) {
    *bytes = max_bytes;
    return IHMC_OK;
  }
  if (*bytes < max_bytes) {
    const uint64_t have = *bytes;
    *bytes = max_bytes;
    return set_error(IHMC_E_INVAL, "checkpoint buffer of %llu bytes, %llu needed", (unsigned long long)have,
                     (unsigned long long)max_bytes);
  }
  std::vector<char> chain, out;
  if (r->state == REQ_RUNNING) {
    // taken by the scheduler at the next round boundary (or from the host copies
    // if the request finishes first)
    r->ckpt_ready = false;
    r->ckpt_wanted = true;
    sv->cv_work.notify_all();
    sv->cv_done.wait(lk, [&] { return r->ckpt_ready || r->state >= REQ_DONE || sv->dead; });
    if (r->ckpt_ready) {
      if (r->ckpt.empty()) return set_error(IHMC_E_DEVICE, "checkpoint of request %llu failed",
                                            (unsigned long long)ticket);
      chain.swap(r->ckpt);
      r->ckpt_ready = false;
    }
  }
  if (r->state == REQ_FAILED) return set_error(IHMC_E_DEVICE, "request %llu failed", (unsigned long long)ticket);
  if (chain.empty() && (r->state == REQ_DONE || r->state == REQ_CANCELLED) && r->st.traj > 0) {
    // retired: its state, field and records are host copies
    uint64_t fh = 0;
    if (r->cd.h_kind == 2) {
      std::vector<double> hp(r->h.size());
      for (size_t i = 0; i < hp.size(); ++i) hp[i] = r->lat.beta * r->h[i];
      fh = field_hash_host(hp.data(), (int64_t)hp.size());
    }
    if ((int64_t)r->psi.size() != r->cd.N)
      return set_error(IHMC_E_DEVICE, "request %llu has no final field", (unsigned long long)ticket);
    chain_checkpoint_host(r->cd, fh, r->st, r->psi.data(), r->rec.data(), (int)r->rec.size(), chain);
  }
  // queued (or retired before any trajectory): the request alone
  served_write(r, chain, out);
  std::memcpy(buf, out.data(), out.size());
  *bytes = out.size();
  return IHMC_OK;
}

extern "C" int ihmc_restore(ihmc_server* sv, const void* buf, uint64_t bytes, uint64_t* ticket) {
  if (!sv || !buf || !ticket) return set_error(IHMC_E_INVAL, "NULL argument");
  SrvHeader h;
  if (bytes < sizeof h) return set_error(IHMC_E_INVAL, "not a served checkpoint (%llu bytes)", (unsigned long long)bytes);
  std::memcpy(&h, buf, sizeof h);
  if (std::memcmp(h.magic, kSrvMagic, 8) != 0 || h.version != kSrvVersion || h.header_bytes != sizeof h)
    return set_error(IHMC_E_INVAL, "not a served checkpoint of this library version");
  if (h.h_len < 0 || h.psi0_len < 0 || h.replay_len < 0 || h.h_len > (int64_t(1) << 33) ||
      h.psi0_len > (int64_t(1) << 33) || h.replay_len > (int64_t(1) << 31))
    return set_error(IHMC_E_INVAL, "served checkpoint is inconsistent");
  const uint64_t prefix = sizeof h + 8 * (uint64_t)h.h_len + 8 * (uint64_t)h.psi0_len + (uint64_t)h.replay_len;
  if (bytes != prefix + h.chain_bytes)
    return set_error(IHMC_E_INVAL, "served checkpoint of %llu bytes, %llu expected", (unsigned long long)bytes,
                     (unsigned long long)(prefix + h.chain_bytes));
  Request* r = new (std::nothrow) Request();
  if (!r) return set_error(IHMC_E_NOMEM, "host allocation failed");
  std::memset(&r->lat, 0, sizeof r->lat);
  std::memset(&r->run, 0, sizeof r->run);
  r->lat.ndim = h.ndim;
  for (int i = 0; i < 3; ++i) r->lat.L[i] = h.L[i];
  r->lat.J = h.J;
  r->lat.beta = h.beta;
  r->lat.C = h.C;
  r->lat.h_len = h.h_len;
  r->run.n_md = h.n_md;
  r->run.n_traj = h.n_traj;
  r->run.traj_len = h.traj_len;
  r->run.integrator = h.integrator;
  r->run.flip_every = h.flip_every;
  r->run.precision = h.precision;
  r->run.n_therm = h.n_therm;
  r->run.form = h.form;
  r->run.seed = h.seed;
  r->run.chain_id = h.chain_id;
  const char* in = (const char*)buf + sizeof h;
  r->h.assign((const double*)in, (const double*)in + h.h_len);
  in += 8 * h.h_len;
  r->psi0.assign((const double*)in, (const double*)in + h.psi0_len);
  in += 8 * h.psi0_len;
  r->replay.assign((const uint8_t*)in, (const uint8_t*)in + h.replay_len);
  in += h.replay_len;
  r->resume.assign(in, in + h.chain_bytes);
  r->lat.h = r->h.empty() ? nullptr : r->h.data();
  int rc = validate(r->lat, r->run, 0);
  if (!rc && r->run.form == FORM_PHI)
    rc = set_error(IHMC_E_UNSUPPORTED, "the server runs psi-form or shifted-form chains");
  const int64_t N = rc ? 0 : lattice_sites(r->lat);
  if (!rc && ((h.psi0_len != 0 && h.psi0_len != N) || (h.replay_len != 0 && h.replay_len != h.n_traj)))
    rc = set_error(IHMC_E_INVAL, "served checkpoint is inconsistent");
  if (rc) {
    delete r;
    return rc;
  }
  return queue_request(sv, r, ticket);
}

extern "C" int ihmc_request_info(ihmc_server* sv, uint64_t ticket, int64_t* out) {
  if (!sv || !out) return set_error(IHMC_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return set_error(IHMC_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
  const Request* r = it->second;
  out[0] = r->state;
  out[1] = lattice_sites(r->lat);
  out[2] = r->run.n_traj;
  out[3] = r->state >= REQ_DONE ? r->st.traj : r->rounds;
  return IHMC_OK;
}

extern "C" int ihmc_poll(ihmc_server* sv, uint64_t ticket, int32_t* state) {
  if (!sv || !state) return set_error(IHMC_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return set_error(IHMC_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
  *state = it->second->state;
  return IHMC_OK;
}

extern "C" int ihmc_wait(ihmc_server* sv, uint64_t ticket, double timeout_s, int32_t* state) {
  if (!sv || !state) return set_error(IHMC_E_INVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return set_error(IHMC_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second;
  sv->cv_done.wait_for(lk, std::chrono::duration<double>(std::max(0.0, timeout_s)),
                       [&] { return r->state >= REQ_DONE; });
  *state = r->state;
  return IHMC_OK;
}

extern "C" int ihmc_fetch(ihmc_server* sv, uint64_t ticket, ihmc_result* out, double* times) {
  if (!sv || !out) return set_error(IHMC_E_INVAL, "NULL argument");
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return set_error(IHMC_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
    r = it->second;
    if (r->state < REQ_DONE) return set_error(IHMC_E_AGAIN, "request %llu is not finished", (unsigned long long)ticket);
    sv->reqs.erase(it);
  }
  if (times) {
    times[0] = r->t_submit;
    times[1] = r->t_admit;
    times[2] = r->t_done;
  }
  int rc = IHMC_OK;
  if (r->state == REQ_CANCELLED) rc = set_error(IHMC_E_CANCELLED, "request %llu was cancelled", (unsigned long long)ticket);
  else if (r->state == REQ_FAILED) rc = set_error(r->err_code ? r->err_code : IHMC_E_DEVICE, "%s", r->error.c_str());
  const int done = (int)r->rec.size();
  for (int t = 0; t < done; ++t) {
    const TrajRecord& q = r->rec[t];
    if (out->dH) out->dH[t] = q.dH;
    if (out->H_old) out->H_old[t] = q.H_old + r->s_off;
    if (out->H_new) out->H_new[t] = q.H_new + r->s_off;
    if (out->m) out->m[t] = q.m;
    if (out->abs_m) out->abs_m[t] = q.abs_m;
    if (out->m2c) out->m2c[t] = q.m2c;
    if (out->beta_eps) out->beta_eps[t] = q.beta_eps;
    if (out->accepted) out->accepted[t] = (q.flags & REC_ACCEPT) ? 1 : 0;
    if (out->flipped) out->flipped[t] = (q.flags & REC_FLIP) ? 1 : 0;
  }
  out->n_traj_done = r->st.traj;
  const int64_t counted = std::max(0, r->st.traj - r->run.n_therm);  // trajectories past thermalisation
  out->acceptance = counted ? (double)r->st.n_acc / (double)counted : 0.0;
  const int64_t nf = counted - r->st.n_nonfinite;
  out->mean_exp_minus_dH = nf > 0 ? r->st.sum_exp_mdh / (double)nf : 0.0;
  out->n_nonfinite = r->st.n_nonfinite;
  out->cg_iterations = r->st.n_cg;
  if (out->psi_final && !r->psi.empty()) {
    std::memcpy(out->psi_final, r->psi.data(), 8 * r->psi.size());
    if (r->delta.size() == r->psi.size())  // a translated request: back to its own coordinates
      for (size_t k = 0; k < r->psi.size(); ++k) out->psi_final[k] -= r->delta[k];
  }
  delete r;
  return rc;
}

extern "C" int ihmc_cancel(ihmc_server* sv, uint64_t ticket) {
  if (!sv) return set_error(IHMC_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return set_error(IHMC_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second;
  auto q = std::find(sv->queue.begin(), sv->queue.end(), r);
  if (r->state == REQ_QUEUED && q != sv->queue.end()) {
    sv->queue.erase(q);
    r->state = REQ_CANCELLED;
    r->t_done = sv->now();
    sv->cv_done.notify_all();
  } else if (r->state <= REQ_RUNNING) {
    r->cancel = true;  // admitted (or being set up): retired at the next round boundary
  }
  return IHMC_OK;
}

extern "C" int ihmc_server_stats(ihmc_server* sv, double* out) {
  if (!sv || !out) return set_error(IHMC_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  out[0] = (double)sv->rounds;
  out[1] = sv->busy_s;
  out[2] = sv->site_steps;
  out[3] = sv->max_seen;
  out[4] = (double)sv->completed;
  out[5] = (double)sv->queue.size();
  out[6] = (double)sv->active.size();
  out[7] = sv->now();
  out[8] = (double)sv->used;
  out[9] = (double)sv->budget;
  return IHMC_OK;
}
