// Autotuner of the lattice tile classes.
//
// Every tile class gives bitwise the same trajectories (sums are formed per
// x-aligned quad of sites and per 4-plane column, then added in exact fixed
// point), so the class is a pure speed choice.  The tuner times the middle
// pass -- the pass a trajectory repeats n_md - 1 times -- of each class on
// replicas of a lattice shape with synthetic fields, and keeps the fastest in
// the context's table; chains take their class from the table when they are
// created.  The table can be saved to and loaded from a JSON file.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <set>
#include <string>
#include <vector>

#include "lattice_kernels.hpp"
#include "runtime_internal.hpp"

namespace ihmc {

// ------------------------------------------------------------------ table ---

TileKey tile_key(const ihmc_lattice& l, int precision) {
  TileKey k;
  k.prec = precision;
  k.ndim = l.ndim;
  k.L0 = l.L[0];
  k.L1 = l.ndim >= 2 ? l.L[1] : 1;
  k.L2 = l.ndim == 3 ? l.L[2] : 1;
  k.site_field = l.h_len > 1 ? 1 : 0;
  return k;
}

int TuneTable::class_for(const TileKey& k) {
  std::lock_guard<std::mutex> lk(mu);
  auto it = m.find(k);
  return it != m.end() ? it->second.cls : tile_class(k.ndim, k.L0, k.L2);
}

static bool key_ok(const TileKey& k) {
  if (k.prec != 4 && k.prec != 8) return false;
  if (k.ndim != 2 && k.ndim != 3) return false;
  const int lim = 1 << 20;
  if (k.L0 < 3 || k.L0 > lim || k.L1 < 3 || k.L1 > lim) return false;
  if (k.ndim == 3 ? (k.L2 < 3 || k.L2 > lim) : k.L2 != 1) return false;
  return k.site_field == 0 || k.site_field == 1;
}

// -------------------------------------------------------- synthetic state ---

// Fields of the timing replicas: values in [-1.5, 1.5) from an integer hash
// of the element index (the pass's cost does not depend on the values).
template <typename T>
__global__ void k_tune_fill(T* a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t h = (uint32_t)i * 0x9E3779B1u + (uint32_t)(i >> 32) * 0x7F4A7C15u;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    a[i] = (T)(((double)h * (1.0 / 4294967296.0) - 0.5) * 3.0);
  }
}

__global__ void k_tune_states(ChainState* st, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  ChainState z;
  memset(&z, 0, sizeof z);
  z.sign = 1;
  st[i] = z;
}

static inline uint64_t r256(uint64_t b) { return (b + 255ull) & ~255ull; }

constexpr int64_t kTuneMinSites = int64_t(1) << 20;  // a launch this large fills the GPU
constexpr int64_t kTuneMaxSites = int64_t(1) << 26;
constexpr int64_t kTuneMaxReplicas = 65536;

// Nanoseconds per site and middle step of every class of key k (timed on the
// two-step launch for 2D when the context fuses steps): replicas of the
// lattice, each with its own fields, `sites` sites in all (the working set the
// choice is for: whether it streams from HBM or stays in the last-level cache
// decides which tile is fastest), one launch over all their tiles.
static int measure_key(ihmc_ctx* ctx, const TileKey& k, int64_t sites, int reps, double* ns) {
  hipStream_t s = ctx->stream;
  ihmc_lattice l{};
  l.ndim = k.ndim;
  l.L[0] = k.L0;
  l.L[1] = k.L1;
  l.L[2] = k.L2;
  l.J = 1.0;
  l.beta = k.ndim == 2 ? 0.44 : 0.22;
  l.C = 2.0 * k.ndim + 0.1;
  const int64_t N = (int64_t)k.L0 * k.L1 * k.L2;
  l.h = nullptr;
  l.h_len = k.site_field ? N : 0;
  ihmc_run r{};
  r.n_md = 20;
  r.n_traj = 1;
  r.traj_len = 1.0;
  r.integrator = IHMC_LEAPFROG;
  r.precision = k.prec;
  ChainDev c0;
  describe_chain(l, r, 0, 0, c0);
  const int64_t R = std::min(kTuneMaxReplicas, std::max<int64_t>(1, (sites + N / 2) / N));
  const int ncls = tile_class_count(k.ndim);
  const uint64_t pb = (uint64_t)k.prec;
  const uint64_t fb =
      r256(((uint64_t)LAT_BUFFERS + (uint64_t)LAT_P_BUFFERS + (uint64_t)k.site_field) * (uint64_t)c0.NP * pb);

  std::vector<std::vector<Tile>> tl(ncls);
  for (int cls = 0; cls < ncls; ++cls) {
    const TileShape ts = tile_shape(k.prec, k.ndim, cls);
    for (int64_t q = 0; q < R; ++q)
      for (int z = 0; z < k.L2; z += (k.ndim == 3 ? ts.bz : 1))
        for (int y = 0; y < k.L1; y += ts.by)
          for (int x = 0; x < k.L0; x += ts.bx) tl[cls].push_back(Tile{(int32_t)q, x, y, z});
  }
  uint64_t total = R * fb + r256(R * sizeof(ChainState)) + r256(R * sizeof(ChainDev));
  for (int cls = 0; cls < ncls; ++cls) total += r256(tl[cls].size() * sizeof(Tile));
  char* blk = (char*)ctx->arena.alloc(total);
  if (!blk)
    return set_error(IHMC_E_NOMEM, "tuning %dD %dx%dx%d needs %llu arena bytes (%llu of %llu in use)", k.ndim, k.L0,
                     k.L1, k.L2, (unsigned long long)total, (unsigned long long)ctx->arena.used,
                     (unsigned long long)ctx->arena.size);
  struct Release {
    ihmc_ctx* ctx;
    void* p;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Release() {
      hipStreamSynchronize(ctx->stream);
      ctx->arena.release(p);
      if (e0) hipEventDestroy(e0);
      if (e1) hipEventDestroy(e1);
    }
  } rel{ctx, blk};

  char* fields = blk;
  ChainState* st = (ChainState*)(fields + R * fb);
  ChainDev* d_cd = (ChainDev*)((char*)st + r256(R * sizeof(ChainState)));
  char* tp = (char*)d_cd + r256(R * sizeof(ChainDev));
  std::vector<Tile*> d_tl(ncls);
  for (int cls = 0; cls < ncls; ++cls) {
    d_tl[cls] = (Tile*)tp;
    tp += r256(tl[cls].size() * sizeof(Tile));
  }

  std::vector<ChainDev> cd(R, c0);
  for (int64_t q = 0; q < R; ++q) {
    char* f = fields + q * fb;
    cd[q].psi = f;
    cd[q].p = f + LAT_BUFFERS * c0.NP * pb;
    cd[q].b = k.site_field ? (const void*)(f + (LAT_BUFFERS + LAT_P_BUFFERS) * c0.NP * pb) : nullptr;
    cd[q].st = st + q;
  }
  const int64_t nel = (int64_t)(R * fb / pb);
  const unsigned fgrid = (unsigned)std::min<int64_t>(4096, (nel + 255) / 256);
  if (k.prec == 4) k_tune_fill<float><<<fgrid, 256, 0, s>>>((float*)fields, nel);
  else k_tune_fill<double><<<fgrid, 256, 0, s>>>((double*)fields, nel);
  HIPCHK(hipGetLastError(), "k_tune_fill");
  k_tune_states<<<(unsigned)((R + 255) / 256), 256, 0, s>>>(st, (int)R);
  HIPCHK(hipGetLastError(), "k_tune_states");
  HIPCHK(hipMemcpyAsync(d_cd, cd.data(), R * sizeof(ChainDev), hipMemcpyHostToDevice, s), "tune chain upload");
  for (int cls = 0; cls < ncls; ++cls)
    HIPCHK(hipMemcpyAsync(d_tl[cls], tl[cls].data(), tl[cls].size() * sizeof(Tile), hipMemcpyHostToDevice, s),
           "tune tile upload");
  HIPCHK(hipEventCreate(&rel.e0), "event");
  HIPCHK(hipEventCreate(&rel.e1), "event");

  // three interleaved rounds over the classes; the minimum of the round means
  double best[kMaxTileClasses];
  for (int cls = 0; cls < kMaxTileClasses; ++cls) best[cls] = NAN;
  const bool pair = (k.ndim == 2) && ctx->fuse_steps;
  const int mode = pair ? PASS_PAIR : PASS_MIDDLE;
  const double steps = pair ? 2.0 : 1.0;
  for (int round = 0; round < 3; ++round) {
    for (int cls = 0; cls < ncls; ++cls) {
      const int nt = (int)tl[cls].size();
      HIPCHK(launch_lattice_pass(k.prec, k.ndim, cls, mode, d_cd, d_tl[cls], nt, 1, 1, s), "tune warm-up");
      HIPCHK(hipEventRecord(rel.e0, s), "event record");
      for (int i = 0; i < reps; ++i)
        HIPCHK(launch_lattice_pass(k.prec, k.ndim, cls, mode, d_cd, d_tl[cls], nt, 1, 1, s), "tune pass");
      HIPCHK(hipEventRecord(rel.e1, s), "event record");
      HIPCHK(hipEventSynchronize(rel.e1), "event sync");
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, rel.e0, rel.e1), "event time");
      const double v = 1e6 * (double)ms / reps / (double)(R * N) / steps;
      if (!(best[cls] <= v)) best[cls] = v;
    }
  }
  for (int cls = 0; cls < kMaxTileClasses; ++cls) ns[cls] = best[cls];
  return IHMC_OK;
}

// Fastest class; the built-in rule's class is kept unless another is faster by
// more than the run-to-run spread of a measurement (3 %).
constexpr double kTuneMargin = 1.03;
static int pick_class(const TileKey& k, const double* ns) {
  const int ncls = tile_class_count(k.ndim);
  int b = 0;
  for (int cls = 1; cls < ncls; ++cls)
    if (ns[cls] < ns[b]) b = cls;
  const int rule = tile_class(k.ndim, k.L0, k.L2);
  return ns[rule] <= kTuneMargin * ns[b] ? rule : b;
}

// ------------------------------------------------------------------ JSON ---

int tune_save(TuneTable& t, const char* path) {
  std::string out = "{\"format\": \"ihmc-tile-classes\", \"version\": 1, \"entries\": [";
  {
    std::lock_guard<std::mutex> lk(t.mu);
    bool first = true;
    char buf[512];
    for (auto& kv : t.m) {
      const TileKey& k = kv.first;
      const TuneEntry& e = kv.second;
      std::snprintf(buf, sizeof buf,
                    "%s\n  {\"precision\": %d, \"ndim\": %d, \"L\": [%d, %d, %d], \"site_field\": %d, "
                    "\"class\": %d, \"source\": %d, \"ns_per_site\": [",
                    first ? "" : ",", k.prec, k.ndim, k.L0, k.L1, k.L2, k.site_field, e.cls, e.source);
      out += buf;
      for (int c = 0; c < kMaxTileClasses; ++c) {
        if (std::isfinite(e.ns_site[c])) std::snprintf(buf, sizeof buf, "%s%.6g", c ? ", " : "", e.ns_site[c]);
        else std::snprintf(buf, sizeof buf, "%snull", c ? ", " : "");
        out += buf;
      }
      out += "]}";
      first = false;
    }
  }
  out += "\n]}\n";
  FILE* f = std::fopen(path, "w");
  if (!f) return set_error(IHMC_E_INVAL, "cannot open %s for writing", path);
  const bool ok = std::fwrite(out.data(), 1, out.size(), f) == out.size();
  if (std::fclose(f) != 0 || !ok) return set_error(IHMC_E_INVAL, "cannot write %s", path);
  return IHMC_OK;
}

// A small JSON reader: objects, arrays, numbers, strings without escapes
// other than \" and \\, true, false, null.
struct JVal {
  enum Kind { NUL, NUM, STR, ARR, OBJ, BOOL } kind = NUL;
  double num = 0.0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal* get(const char* key) const {
    for (auto& kv : obj)
      if (kv.first == key) return &kv.second;
    return nullptr;
  }
};

struct JParser {
  const char* p;
  const char* end;
  int depth = 0;
  void ws() {
    while (p < end && (*p == ' ' || *p == '\n' || *p == '\t' || *p == '\r')) ++p;
  }
  bool lit(const char* s) {
    const size_t n = std::strlen(s);
    if ((size_t)(end - p) < n || std::strncmp(p, s, n) != 0) return false;
    p += n;
    return true;
  }
  bool string(std::string& out) {
    if (p >= end || *p != '"') return false;
    ++p;
    while (p < end && *p != '"') {
      if (*p == '\\') {
        ++p;
        if (p >= end || (*p != '"' && *p != '\\')) return false;
      }
      out += *p++;
    }
    if (p >= end) return false;
    ++p;
    return true;
  }
  bool value(JVal& v) {
    if (++depth > 16) return false;
    ws();
    bool ok = false;
    if (p >= end) {
      ok = false;
    } else if (*p == '{') {
      v.kind = JVal::OBJ;
      ++p;
      ws();
      if (p < end && *p == '}') {
        ++p;
        ok = true;
      } else {
        while (true) {
          ws();
          std::string key;
          if (!string(key)) break;
          ws();
          if (p >= end || *p != ':') break;
          ++p;
          JVal x;
          if (!value(x)) break;
          v.obj.emplace_back(key, std::move(x));
          ws();
          if (p < end && *p == ',') {
            ++p;
            continue;
          }
          if (p < end && *p == '}') {
            ++p;
            ok = true;
          }
          break;
        }
      }
    } else if (*p == '[') {
      v.kind = JVal::ARR;
      ++p;
      ws();
      if (p < end && *p == ']') {
        ++p;
        ok = true;
      } else {
        while (true) {
          JVal x;
          if (!value(x)) break;
          v.arr.push_back(std::move(x));
          ws();
          if (p < end && *p == ',') {
            ++p;
            continue;
          }
          if (p < end && *p == ']') {
            ++p;
            ok = true;
          }
          break;
        }
      }
    } else if (*p == '"') {
      v.kind = JVal::STR;
      ok = string(v.str);
    } else if (lit("null")) {
      v.kind = JVal::NUL;
      ok = true;
    } else if (lit("true")) {
      v.kind = JVal::BOOL;
      v.num = 1.0;
      ok = true;
    } else if (lit("false")) {
      v.kind = JVal::BOOL;
      ok = true;
    } else {
      char* q = nullptr;
      const std::string tok(p, (size_t)std::min<ptrdiff_t>(end - p, 64));
      v.num = std::strtod(tok.c_str(), &q);
      if (q != tok.c_str()) {
        v.kind = JVal::NUM;
        p += q - tok.c_str();
        ok = true;
      }
    }
    --depth;
    return ok;
  }
};

static bool get_int(const JVal& o, const char* key, int32_t& out) {
  const JVal* v = o.get(key);
  if (!v || v->kind != JVal::NUM || v->num != std::floor(v->num) || std::fabs(v->num) > 1e9) return false;
  out = (int32_t)v->num;
  return true;
}

int tune_load(TuneTable& t, const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return set_error(IHMC_E_INVAL, "cannot open %s", path);
  std::string text;
  char buf[65536];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  std::fclose(f);
  JParser jp{text.data(), text.data() + text.size()};
  JVal root;
  bool ok = jp.value(root);
  jp.ws();
  if (!ok || jp.p != jp.end || root.kind != JVal::OBJ) return set_error(IHMC_E_INVAL, "%s: not a JSON object", path);
  const JVal* fmt = root.get("format");
  if (!fmt || fmt->kind != JVal::STR || fmt->str != "ihmc-tile-classes")
    return set_error(IHMC_E_INVAL, "%s: not a tile-class table", path);
  const JVal* ents = root.get("entries");
  if (!ents || ents->kind != JVal::ARR) return set_error(IHMC_E_INVAL, "%s: no entries array", path);
  std::vector<std::pair<TileKey, TuneEntry>> got_entries;
  for (size_t i = 0; i < ents->arr.size(); ++i) {
    const JVal& e = ents->arr[i];
    TileKey k{};
    TuneEntry te;
    const JVal* L = e.kind == JVal::OBJ ? e.get("L") : nullptr;
    bool good = e.kind == JVal::OBJ && get_int(e, "precision", k.prec) && get_int(e, "ndim", k.ndim) &&
                get_int(e, "site_field", k.site_field) && get_int(e, "class", te.cls) &&
                get_int(e, "source", te.source) && L && L->kind == JVal::ARR && L->arr.size() == 3;
    if (good) {
      int32_t* dst[3] = {&k.L0, &k.L1, &k.L2};
      for (int d = 0; d < 3; ++d) {
        const JVal& x = L->arr[d];
        if (x.kind != JVal::NUM || x.num != std::floor(x.num) || std::fabs(x.num) > 1e9) good = false;
        else *dst[d] = (int32_t)x.num;
      }
    }
    good = good && key_ok(k) && te.cls >= 0 && te.cls < tile_class_count(k.ndim) &&
           (te.source == IHMC_TUNE_MEASURED || te.source == IHMC_TUNE_PINNED);
    for (int c = 0; c < kMaxTileClasses; ++c) te.ns_site[c] = NAN;
    const JVal* ns = good ? e.get("ns_per_site") : nullptr;
    if (ns && ns->kind == JVal::ARR)
      for (size_t c = 0; c < ns->arr.size() && c < (size_t)kMaxTileClasses; ++c)
        if (ns->arr[c].kind == JVal::NUM) te.ns_site[c] = ns->arr[c].num;
    if (!good) return set_error(IHMC_E_INVAL, "%s: entry %zu is malformed or out of range", path, i);
    got_entries.emplace_back(k, te);
  }
  std::lock_guard<std::mutex> lk(t.mu);
  for (auto& kv : got_entries) t.m[kv.first] = kv.second;
  return IHMC_OK;
}

}  // namespace ihmc

using namespace ihmc;

// ================================================================= C ABI ===

extern "C" int ihmc_tile_shape(int32_t ndim, int32_t cls, int32_t* out, int32_t* n_classes) {
  if (ndim != 2 && ndim != 3) return set_error(IHMC_E_INVAL, "ndim must be 2 or 3");
  if (n_classes) *n_classes = tile_class_count(ndim);
  if (!out) return IHMC_OK;
  if (cls < 0 || cls >= tile_class_count(ndim))
    return set_error(IHMC_E_INVAL, "tile class %d does not exist for %dD", cls, ndim);
  const TileShape ts = tile_shape(4, ndim, cls);
  out[0] = ts.bx;
  out[1] = ts.by;
  out[2] = ndim == 3 ? ts.bz : 1;
  return IHMC_OK;
}

extern "C" int ihmc_tune(ihmc_ctx* ctx, int32_t n, const ihmc_lattice* lats, const int32_t* precision, int64_t sites,
                         int32_t reps, int32_t flags, int32_t* n_measured) {
  CTX_OK(ctx);
  if (n_measured) *n_measured = 0;
  if (n < 0 || (n > 0 && (!lats || !precision))) return set_error(IHMC_E_INVAL, "bad lattice arrays");
  if (reps < 0 || reps > 10000) return set_error(IHMC_E_INVAL, "reps must be in [0, 10000]");
  if (sites < 0) return set_error(IHMC_E_INVAL, "sites must be >= 0");
  if (flags & ~IHMC_TUNE_FORCE) return set_error(IHMC_E_INVAL, "unknown flags 0x%x", flags);
  std::set<TileKey> keys;
  int64_t total = 0;
  for (int i = 0; i < n; ++i) {
    ihmc_run r{};
    r.n_md = 1;
    r.traj_len = 1.0;
    r.precision = precision[i];
    const int rc = validate(lats[i], r, i);
    if (rc) return rc;
    keys.insert(tile_key(lats[i], precision[i]));
    total += lattice_sites(lats[i]);
  }
  if (sites == 0) sites = total;
  sites = std::min(kTuneMaxSites, std::max(kTuneMinSites, sites));
  if (reps == 0) reps = sites > (int64_t(1) << 23) ? 4 : 10;
  int measured = 0;
  for (const TileKey& k : keys) {
    {
      std::lock_guard<std::mutex> lk(ctx->tune.mu);
      auto it = ctx->tune.m.find(k);
      if (it != ctx->tune.m.end() &&
          (it->second.source == IHMC_TUNE_PINNED || !(flags & IHMC_TUNE_FORCE)))
        continue;
    }
    double ns[kMaxTileClasses];
    const int rc = measure_key(ctx, k, sites, reps, ns);
    if (rc) return rc;
    TuneEntry e;
    for (int c = 0; c < kMaxTileClasses; ++c) e.ns_site[c] = ns[c];
    e.cls = pick_class(k, ns);
    e.source = IHMC_TUNE_MEASURED;
    {
      std::lock_guard<std::mutex> lk(ctx->tune.mu);
      ctx->tune.m[k] = e;
    }
    ++measured;
    if (n_measured) *n_measured = measured;
  }
  const char* cache = std::getenv("IHMC_TUNE_CACHE");
  if (measured > 0 && cache && *cache) return tune_save(ctx->tune, cache);
  return IHMC_OK;
}

extern "C" int ihmc_tune_lookup(ihmc_ctx* ctx, const ihmc_lattice* lat, int32_t precision, int32_t* cls,
                                int32_t* source, double* ns_site) {
  if (!ctx || !lat || !cls) return set_error(IHMC_E_INVAL, "NULL argument");
  ihmc_run r{};
  r.n_md = 1;
  r.traj_len = 1.0;
  r.precision = precision;
  const int rc = validate(*lat, r, 0);
  if (rc) return rc;
  const TileKey k = tile_key(*lat, precision);
  std::lock_guard<std::mutex> lk(ctx->tune.mu);
  auto it = ctx->tune.m.find(k);
  if (it == ctx->tune.m.end()) {
    *cls = tile_class(k.ndim, k.L0, k.L2);
    if (source) *source = IHMC_TUNE_RULE;
    if (ns_site)
      for (int c = 0; c < kMaxTileClasses; ++c) ns_site[c] = NAN;
  } else {
    *cls = it->second.cls;
    if (source) *source = it->second.source;
    if (ns_site)
      for (int c = 0; c < kMaxTileClasses; ++c) ns_site[c] = it->second.ns_site[c];
  }
  return IHMC_OK;
}

extern "C" int ihmc_tune_pin(ihmc_ctx* ctx, const ihmc_lattice* lat, int32_t precision, int32_t cls) {
  if (!ctx || !lat) return set_error(IHMC_E_INVAL, "NULL argument");
  ihmc_run r{};
  r.n_md = 1;
  r.traj_len = 1.0;
  r.precision = precision;
  const int rc = validate(*lat, r, 0);
  if (rc) return rc;
  const TileKey k = tile_key(*lat, precision);
  if (cls >= tile_class_count(k.ndim)) return set_error(IHMC_E_INVAL, "tile class %d does not exist for %dD", cls, k.ndim);
  std::lock_guard<std::mutex> lk(ctx->tune.mu);
  if (cls < 0) {
    ctx->tune.m.erase(k);
    return IHMC_OK;
  }
  TuneEntry e;
  auto it = ctx->tune.m.find(k);
  for (int c = 0; c < kMaxTileClasses; ++c) e.ns_site[c] = it != ctx->tune.m.end() ? it->second.ns_site[c] : NAN;
  e.cls = cls;
  e.source = IHMC_TUNE_PINNED;
  ctx->tune.m[k] = e;
  return IHMC_OK;
}

extern "C" int ihmc_tune_save(ihmc_ctx* ctx, const char* path) {
  if (!ctx || !path) return set_error(IHMC_E_INVAL, "NULL argument");
  return tune_save(ctx->tune, path);
}

extern "C" int ihmc_tune_load(ihmc_ctx* ctx, const char* path) {
  if (!ctx || !path) return set_error(IHMC_E_INVAL, "NULL argument");
  return tune_load(ctx->tune, path);
}

extern "C" int ihmc_tune_check(const char* path, int32_t* n_entries) {
  if (!path) return set_error(IHMC_E_INVAL, "NULL argument");
  TuneTable t;
  const int rc = tune_load(t, path);
  if (rc) return rc;
  if (n_entries) *n_entries = (int32_t)t.m.size();
  return IHMC_OK;
}
