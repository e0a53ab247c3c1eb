// Host side of the MI355X block-multiresolution solver: forest manager (keys,
// Morton order, neighbour relations, validation), plans for refinement and
// coarsening (completeness + gradedness fixed point), descriptor upload and the
// C ABI declared in include/mrb.h.
#include "../../include/mrb.h"
#include "internal.hpp"
#include "mlp.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace mrb;

namespace {

struct Leaf {
  int level;
  int c[3];
  int slot;
  uint64_t morton;
};

inline uint64_t pack_key(int l, const int* c) {
  return ((uint64_t)l << 60) | (uint64_t)(uint32_t)c[0] | ((uint64_t)(uint32_t)c[1] << 20) |
         ((uint64_t)(uint32_t)c[2] << 40);
}

inline int wrapi(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// Leaf position by key (level, coords).  A dense table with one cell per possible
// block of every level when that fits in 2^24 cells (a lookup is one load; clearing
// touches only the cells set), else a hash map.
struct LeafIndex {
  int dim = 2, jmax = 0;
  bool dense = false;
  std::vector<int> cells;
  std::vector<size_t> off, used;
  std::unordered_map<uint64_t, int> map;
  size_t n = 0;
  void init(int d, int jm) {
    dim = d;
    jmax = jm;
    off.assign(jm + 2, 0);
    size_t tot = 0;
    for (int l = 1; l <= jm && tot <= ((size_t)1 << 24); ++l) {
      off[l] = tot;
      tot += (size_t)1 << (d * l);
    }
    dense = tot <= ((size_t)1 << 24);
    cells.assign(dense ? tot : 0, -1);
    used.clear();
    map.clear();
    n = 0;
  }
  bool valid(uint64_t key) const {
    const int l = (int)(key >> 60);
    if (l < 1 || l > jmax) return false;
    const uint64_t lim = (uint64_t)1 << l;
    return (key & 0xFFFFF) < lim && ((key >> 20) & 0xFFFFF) < lim && (dim > 2 ? ((key >> 40) & 0xFFFFF) < lim
                                                                                : ((key >> 40) & 0xFFFFF) == 0);
  }
  size_t cell(uint64_t key) const {
    const int l = (int)(key >> 60);
    return off[l] + (key & 0xFFFFF) + (((key >> 20) & 0xFFFFF) << l) + (((key >> 40) & 0xFFFFF) << (2 * l));
  }
  void clear() {
    if (dense) {
      for (size_t u : used) cells[u] = -1;
      used.clear();
    } else {
      map.clear();
    }
    n = 0;
  }
  void reserve(size_t k) {
    if (dense) used.reserve(k);
    else map.reserve(k * 2);
  }
  void set(uint64_t key, int i) {
    if (dense) {
      const size_t u = cell(key);
      if (cells[u] < 0) {
        used.push_back(u);
        ++n;
      }
      cells[u] = i;
    } else {
      auto r = map.emplace(key, i);
      if (r.second) ++n;
      else r.first->second = i;
    }
  }
  int find(uint64_t key) const {
    if (!valid(key)) return -1;
    if (dense) return cells[cell(key)];
    auto it = map.find(key);
    return it == map.end() ? -1 : it->second;
  }
  size_t size() const { return n; }
};

// Host worker threads kept for the life of a context (spawning threads per plan costs
// more than the work they would share).  run(n, f) calls f(0..n-1), f(0) on the caller.
struct WorkerPool {
  std::vector<std::thread> th;
  std::mutex m;
  std::condition_variable cv, done_cv;
  std::function<void(int)> job;
  int njobs = 0, next = 1, pending = 0;
  long gen = 0;
  bool stop = false;
  ~WorkerPool() {
    {
      std::lock_guard<std::mutex> g(m);
      stop = true;
    }
    cv.notify_all();
    for (auto& t : th) t.join();
  }
  void ensure(int nthreads) {
    while ((int)th.size() < nthreads) th.emplace_back([this] { loop(); });
  }
  void loop() {
    long seen = 0;
    for (;;) {
      int j;
      {
        std::unique_lock<std::mutex> g(m);
        cv.wait(g, [&] { return stop || (gen != seen && next < njobs); });
        if (stop) return;
        j = next++;
        if (next >= njobs) seen = gen;
      }
      job(j);
      {
        std::lock_guard<std::mutex> g(m);
        if (--pending == 0) done_cv.notify_all();
      }
    }
  }
  void run(int n, const std::function<void(int)>& f) {
    if (n <= 1) {
      f(0);
      return;
    }
    ensure(n - 1);
    {
      std::lock_guard<std::mutex> g(m);
      job = f;
      njobs = n;
      next = 1;
      pending = n - 1;
      ++gen;
    }
    cv.notify_all();
    f(0);
    std::unique_lock<std::mutex> g(m);
    done_cv.wait(g, [&] { return pending == 0; });
  }
};

// Pinned host staging buffer; an event guards reuse while a copy is in flight.
struct Staging {
  void* h = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};

}  // namespace

struct mrb_ctx {
  mrb_config cfg;
  Shape shape;
  int np = 0;
  size_t bsz = 0;  // nf * np
  hipStream_t stream = nullptr;
  double* u = nullptr;
  double* unew = nullptr;
  void* k[3] = {nullptr, nullptr, nullptr};
  std::vector<double> thr, off;

  std::vector<Leaf> leaves;                  // forest order
  LeafIndex index;                           // key -> position in leaves
  std::vector<int> free_slots;
  bool have_forest = false, have_data = false;

  std::vector<BlockDesc> hblk;
  std::vector<NbEntry> hnb;
  std::vector<int> hlist, level_off;         // blocks grouped by level (plain form)
  std::vector<NbEntry> hnb_next;             // descriptor build buffers, reused
  std::vector<std::vector<NbEntry>> desc_parts;
  WorkerPool pool;
  long desc_thread_min = 256;                // forests at least this large use host threads

  char* arena = nullptr;        // packed topology in use: header, blocks, entries, lists, plans
  TopoHeader arena_hdr{};       // its header (kernels take it by value)
  char* work_arena = nullptr;   // the arena uploads go to (owned)
  size_t arena_cap = 0, arena_bytes = 0;
  // memo of topology transitions on small forests: a refine-all or a coarsening from a
  // state seen before (same leaves, slots, free-list tail and flags) reuses the host
  // plan and a device copy of its packed topology instead of planning and uploading
  struct Memo {
    int kind = 0;                       // 0 refine-all, 1 coarsen
    std::vector<int> material;          // leaves, free-list tail and flags the plan came from
    long last_use = 0;
    std::vector<Leaf> leaves;
    std::vector<BlockDesc> hblk;
    std::vector<NbEntry> hnb;
    std::vector<int> hlist, level_off;
    size_t pop = 0;                     // free slots taken from the back
    std::vector<int> pushed;            // slots returned, in order
    int pending_ref = 0, nfam = 0, npar = 0;
    char* arena = nullptr;
    TopoHeader hdr{};
    size_t arena_bytes = 0;
    const int* smap = nullptr;          // coarsenings: the arena's speculation map, or null
  };
  std::vector<Memo> memo;
  long memo_clock = 0, memo_hits = 0;
  int8_t* dflags = nullptr;     // device views of h_flags / h_maxd (mapped host memory)
  double* dmaxd = nullptr;
  unsigned long long* dacc = nullptr;   // analysis partial maxima (zero between passes)
  int* ddone = nullptr;                 // analysis sub-tiles finished (zero between passes)
  double* ds2 = nullptr;
  double* ds = nullptr;
  double* dghost = nullptr;
  double* dscratch = nullptr;
  size_t scratch_cap = 0;
  int* dslots = nullptr;

  Staging st_topo[2], st_slots;
  int st_cur = 0;
  int8_t* h_flags = nullptr;   // pinned, mapped
  double* h_maxd = nullptr;    // pinned, mapped
  // a second mapped set, written by the speculative second analysis of an adapt
  int8_t *h_flags2 = nullptr, *dflags2 = nullptr;
  // whole-sweep launches: barrier words (device) and the time-out word (mapped host)
  unsigned* dbar = nullptr;
  int *h_err = nullptr, *d_err = nullptr;
  int sweep_mode = 2;          // 0 four launches, 1 one launch with grid barriers, 2 the autotuner's choice,
                               // 3 overlapped-tile RK4 where the forest is on one level
  bool sweep_one_tuned = false;
  int rk4t_nsub = 0;           // overlapped-tile RK4: tuned sub-tiles per axis (0: not tuned)
  bool rk4t_tuned = false;     // the autotuner found it faster than the stage launches
  int ana_nsub = 0;            // first analysis folded into it: tiling (0 not tuned: the RK4 tiling;
  int ana_tpb = 256;           // -1: not folded) and threads per workgroup
  int ref_fold = 1;            // the safety-zone refinement folded in as well (0: the autotuner found
                               // the refinement launch before it faster)
  int ref_nsub = 0;            // its tiling and threads per workgroup (0: those of the folded analysis)
  int ref_tpb = 256;
  int ma_nsub = 0;             // with the speculated coarsening's second analysis folded in as well:
  int ma_tpb = 256;            // tiling and threads (0: those of the folded refinement)
  int sweep_grid = 0;          // workgroups of the last whole-sweep launch
  double *h_maxd2 = nullptr, *dmaxd2 = nullptr;
  double *h_mq = nullptr, *dmq = nullptr;   // mothers' detail maxima per child sub-tile (folded second analysis)
  // second bank of the first pass's flags and maxima and of the mothers' shares (queued
  // steps alternate between the banks), and the events the queued steps are waited on
  int8_t *h_flags_b = nullptr, *dflags_b = nullptr;
  double *h_maxd_b = nullptr, *dmaxd_b = nullptr;
  double *h_mq_b = nullptr, *dmq_b = nullptr;
  hipEvent_t ev_issue[2] = {nullptr, nullptr};
  long n_queued = 0, n_taken_back = 0;      // steps launched ahead of the previous read-back; taken back
  int mq_parts = 0;                         // sub-tiles per block of the last folded second analysis
  // a tile launch with sub-tiles and the first analysis folded in leaves each sub-tile's
  // maximum |detail| here (mapped; two banks like the flags), for the host to combine
  struct PartState {
    int parts = 0, n = 0, level = 0;   // parts 0: nothing to combine
  };
  double *h_part = nullptr, *dpart = nullptr, *h_part_b = nullptr, *dpart_b = nullptr;
  PartState part_st, part_st_b;
  int flag_set = 0;                    // set the next analysis writes
  std::vector<int8_t> spec_flags;      // first-pass flags of the last adapt
  long spec_hits = 0, spec_misses = 0;
  int ncu = 256;
  int nsub = 0;                // stage sub-tiles per axis (0 = choose by block count)
  int tpb = 256;               // stage threads per workgroup (for the tuned nsub)
  int nsub_mr = -1;            // analysis sub-tiles per axis (-1 = whole blocks, measured best)
  int tpb_mr = 256;            // analysis threads per workgroup for whole blocks (tuned)
  int nsub_ref = 0;            // refinement sub-tiles per axis (0 = choose by work count)
  int order = 0;               // stage processing order: 0 forest (Morton), 1 level-sorted
  std::string tune_log;
  // captured step graphs (refine, four stages, first analysis), keyed by launch parameters
  bool use_graph = true;
  // graph mode: 0 off, 1 on, 2 automatic (steps alternate between the two launch
  // paths until each has ten samples, then the faster median wall time wins)
  int graph_mode = 2;
  std::vector<double> probe_us[2];
  struct GraphEntry { uint64_t key[7 + sizeof(TopoHeader) / 8]; hipGraphExec_t exec; };
  std::vector<GraphEntry> graphs;
  long n_graph_launches = 0;
  // host-side time (microseconds) by phase
  double hus_refine_plan = 0, hus_coarsen_plan = 0, hus_upload = 0, hus_wait = 0, hus_launch = 0;
  double hus_index = 0, hus_desc = 0, hus_fixed = 0;   // parts of the plans: ordering, entries, fixed point
  double hus_desc_par = 0;                              // entries: the per-block (threaded) part
  // learned predictor: model, Adam state and batch workspace (device)
  int mlp_nin = 0, mlp_np = 0, mlp_t = 0, mlp_cap = 0;
  float *mp = nullptr, *mgrad = nullptr, *mm = nullptr, *mv = nullptr, *mnorm = nullptr;
  float *mx = nullptr, *mxn = nullptr, *mz1 = nullptr, *ma1 = nullptr, *mz2 = nullptr, *ma2 = nullptr;
  float *mlog = nullptr, *mloss = nullptr, *mdl = nullptr, *mdz1 = nullptr, *mdz2 = nullptr, *mcw = nullptr;
  float* mpmax = nullptr;
  int8_t *my = nullptr, *mpred = nullptr;
  int pending_ref = 0;          // parents in the last uploaded refinement plan
  bool hcount_ref_zero = true;  // the uploaded header has no refinement plan

  LevelTab lt;
  Physics ph;
  int grid = 2048;

  std::vector<int8_t> last_flags;     // capacity reserved for max_blocks at create
  std::vector<double> last_maxd;
  bool have_flags = false;
  // the library's static device scratch on this context's GPU (mrb_mr_pass_noalloc)
  void* scratch_dev = nullptr;
  std::string scratch_err;
  // Device-resident topology (topo.hip): the step's refinement and coarsening plans and
  // neighbour entries are built on the device; the host forest above is brought up to
  // date (pulled) only when an entry point other than mrb_step needs it.
  struct DevTopo {
    bool ready = false;          // buffers allocated
    bool active = false;         // the device holds the current grid (host copy stale)
    bool unavailable = false;    // the dense index would not fit
    int mode = 2;                // 0 host planning, 1 device, 2 device when the refined grid exceeds
                                 // the memo limit (host plans are memoised below it)
    char* arena[2] = {nullptr, nullptr};
    size_t arena_bytes = 0;
    int cur = 0;
    int stride = 0;              // entry row stride: the most entries a block can have
    int* cells = nullptr;
    size_t ncells = 0;
    int cell_off[kMaxLevels + 1];
    int* stack = nullptr;        // free pool slots
    int* scratch = nullptr;      // [3 * max_blocks]
    int* edges = nullptr;        // coarsening plan: edge count, family count, edges
    int* err = nullptr;          // device error word
    int8_t* flags = nullptr;     // analysis flags and maxima of the device path
    double* maxd = nullptr;
    int* h_out = nullptr;        // mapped counts written by the plan kernels
    int* d_out = nullptr;
    int n = 0, top = 0;
    long hist[kMaxLevels];
    bool have_flags = false;     // flags/maxd above describe the current grid
    Staging st_blk, st_stack;
    long steps = 0, passes = 0, pushes = 0, pulls = 0;
  } dev;

  // statistics
  long n_steps = 0, n_rk4 = 0, n_block_updates = 0, n_mr = 0, n_fam = 0, n_refined = 0;
  // kernel timing: event pairs per kernel kind, resolved in mrb_stats
  bool timing = false;
  struct Timed { int kind; hipEvent_t a, b; double bytes; int count; };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> ev_pool;
  double t_ms[16] = {};
  double t_bytes[16] = {};
  long t_launches[16] = {};
  std::string err;
};

namespace {

double now_us() {
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// adds the elapsed host time of a scope to an accumulator
struct HostTimer {
  double* acc;
  double t0;
  explicit HostTimer(double* a) : acc(a), t0(now_us()) {}
  ~HostTimer() { *acc += now_us() - t0; }
};

mrb_status fail(mrb_ctx* c, mrb_status s, const std::string& m) {
  c->err = m;
  return s;
}

// kernel kinds for timing
enum { T_STAGE = 0, T_GHOST = 1, T_RHS_PLAIN = 2, T_MR = 3, T_REFINE = 4, T_COARSEN = 5, T_READ = 6, T_TOPO = 7,
       T_FILTER = 8, T_RK4T = 9, T_NKIND = 10 };
const char* kKindName[T_NKIND] = {"stage", "ghost", "rhs_plain", "mr", "refine", "coarsen", "read", "topology",
                                  "filter", "rk4_tile"};

hipEvent_t take_event(mrb_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Bracket one launch with events when timing is on; `bytes` are the algorithmic
// bytes the launch moves.
// One event pair around `count` back-to-back launches of one kernel kind (count > 1
// for the four stage launches of a sweep, so the pair's own overhead is paid once).
struct TimeScope {
  mrb_ctx* c;
  int kind;
  double bytes;
  int count;
  hipEvent_t a = nullptr;
  TimeScope(mrb_ctx* c_, int k, double b, int n = 1, bool on = true) : c(c_), kind(k), bytes(b), count(n) {
    if (on && c->timing && (a = take_event(c))) (void)hipEventRecord(a, c->stream);
  }
  ~TimeScope() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) { c->ev_pool.push_back(a); return; }
    (void)hipEventRecord(b, c->stream);
    c->timed.push_back(mrb_ctx::Timed{kind, a, b, bytes, count});
  }
};

void resolve_timing(mrb_ctx* c) {
  if (c->timed.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& t : c->timed) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      c->t_ms[t.kind] += ms;
      c->t_bytes[t.kind] += t.bytes;
      c->t_launches[t.kind] += t.count;
    }
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->timed.clear();
}

#define HIPCHK(ctx, call)                                                                          \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return fail(ctx, MRB_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));           \
  } while (0)

// spread the low 21 bits of v to every third bit (3D) / the low 32 bits to every
// second bit (2D)
inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}
inline uint64_t spread2(uint64_t v) {
  v &= 0xffffffffULL;
  v = (v | v << 16) & 0x0000ffff0000ffffULL;
  v = (v | v << 8) & 0x00ff00ff00ff00ffULL;
  v = (v | v << 4) & 0x0f0f0f0f0f0f0f0fULL;
  v = (v | v << 2) & 0x3333333333333333ULL;
  v = (v | v << 1) & 0x5555555555555555ULL;
  return v;
}

// Morton key of coords << (jmax - l), x least significant
uint64_t morton_of(const mrb_ctx* c, int l, const int* co) {
  const int sh = c->cfg.jmax - l;
  if (c->cfg.dim == 2)
    return spread2((uint64_t)co[0] << sh) | spread2((uint64_t)co[1] << sh) << 1;
  return spread3((uint64_t)co[0] << sh) | spread3((uint64_t)co[1] << sh) << 1 | spread3((uint64_t)co[2] << sh) << 2;
}

mrb_status stage_upload(mrb_ctx* c, Staging& s, const void* src, size_t bytes, void* dst) {
  if (bytes == 0) return MRB_OK;
  if (s.pending) {
    HIPCHK(c, hipEventSynchronize(s.ev));
    s.pending = false;
  }
  if (!s.ev) HIPCHK(c, hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
  if (bytes > s.cap) {
    if (s.h) HIPCHK(c, hipHostFree(s.h));
    s.h = nullptr;
    size_t cap = std::max(bytes, (size_t)4096);
    HIPCHK(c, hipHostMalloc(&s.h, cap, hipHostMallocDefault));
    s.cap = cap;
  }
  std::memcpy(s.h, src, bytes);
  HIPCHK(c, hipMemcpyAsync(dst, s.h, bytes, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipEventRecord(s.ev, c->stream));
  s.pending = true;
  return MRB_OK;
}

void release_staging(Staging& s) {
  if (s.pending) (void)hipEventSynchronize(s.ev);
  if (s.h) (void)hipHostFree(s.h);
  if (s.ev) (void)hipEventDestroy(s.ev);
  s = Staging();
}

void sort_and_index(mrb_ctx* c) {
  HostTimer ht(&c->hus_index);
  for (auto& L : c->leaves) L.morton = morton_of(c, L.level, L.c);
  std::sort(c->leaves.begin(), c->leaves.end(), [](const Leaf& a, const Leaf& b) { return a.morton < b.morton; });
  c->index.clear();
  c->index.reserve(c->leaves.size());
  for (size_t i = 0; i < c->leaves.size(); ++i) c->index.set(pack_key(c->leaves[i].level, c->leaves[i].c), (int)i);
}

const Leaf* find_leaf(const mrb_ctx* c, int l, const int* co) {
  if (l < 1 || l > c->cfg.jmax) return nullptr;
  int w[3] = {0, 0, 0};
  for (int a = 0; a < c->cfg.dim; ++a) w[a] = wrapi(co[a], 1 << l);
  const int i = c->index.find(pack_key(l, w));
  return i < 0 ? nullptr : &c->leaves[i];
}

// Neighbour entries of leaf i appended to out (nb_begin relative to out's start);
// returns an error message, or nullptr, if the forest is not graded around it.
const char* block_entries(const mrb_ctx* c, int i, std::vector<NbEntry>& out, BlockDesc& B,
                          std::vector<NbEntry>& co, std::vector<NbEntry>& sa, std::vector<NbEntry>& fi) {
  const int d = c->cfg.dim, bs = c->cfg.bs, jmax = c->cfg.jmax;
  const Leaf& L = c->leaves[i];
  co.clear();
  sa.clear();
  fi.clear();
  sa.push_back(NbEntry{L.slot, 0, {0, 0, 0}});
  auto add = [](std::vector<NbEntry>& v, const NbEntry& e) {
    for (auto& x : v)
      if (x.slot == e.slot && x.o[0] == e.o[0] && x.o[1] == e.o[1] && x.o[2] == e.o[2]) return;
    v.push_back(e);
  };
  const int nd = d == 2 ? 9 : 27;
  for (int q = 0; q < nd; ++q) {
    int dlt[3] = {q % 3 - 1, (q / 3) % 3 - 1, d > 2 ? q / 9 - 1 : 0};
    if (dlt[0] == 0 && dlt[1] == 0 && dlt[2] == 0) continue;
    int cn[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) cn[a] = L.c[a] + dlt[a];
    if (const Leaf* s = find_leaf(c, L.level, cn)) {
      // origins differ between directions, so a same-level entry is never repeated
      NbEntry e{s->slot, 0, {0, 0, 0}};
      for (int a = 0; a < d; ++a) e.o[a] = (int8_t)(dlt[a] * (bs - 1));
      sa.push_back(e);
      continue;
    }
    int pc[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) pc[a] = cn[a] >> 1;  // floor division
    if (L.level > 1) {
      if (const Leaf* s = find_leaf(c, L.level - 1, pc)) {
        NbEntry e{s->slot, -1, {0, 0, 0}};
        for (int a = 0; a < d; ++a) e.o[a] = (int8_t)((2 * pc[a] - L.c[a]) * (bs - 1));
        add(co, e);
        continue;
      }
    }
    if (L.level >= jmax) return "forest is not graded or leaves a hole next to a level-jmax block";
    // the region is split: its children touching this block must all be leaves
    int nb = 1 << d;
    for (int b = 0; b < nb; ++b) {
      int beta[3] = {0, 0, 0};
      bool ok = true;
      for (int a = 0; a < d; ++a) {
        beta[a] = (b >> a) & 1;
        if (dlt[a] == 1 && beta[a] != 0) ok = false;
        if (dlt[a] == -1 && beta[a] != 1) ok = false;
      }
      if (!ok) continue;
      int ch[3] = {0, 0, 0};
      for (int a = 0; a < d; ++a) ch[a] = 2 * wrapi(cn[a], 1 << L.level) + beta[a];
      const Leaf* s = find_leaf(c, L.level + 1, ch);
      if (!s) return "forest is not graded (a neighbour differs by two or more levels)";
      // (direction, child) pairs give distinct origins: no repeats either
      NbEntry e{s->slot, 1, {0, 0, 0}};
      for (int a = 0; a < d; ++a) e.o[a] = (int8_t)(dlt[a] * (bs - 1) + beta[a] * ((bs - 1) / 2));
      fi.push_back(e);
    }
  }
  B.slot = L.slot;
  B.level = L.level;
  for (int a = 0; a < 3; ++a) B.c[a] = L.c[a];
  B.nb_begin = (int)out.size();
  B.n_ent = (int)(co.size() + sa.size() + fi.size());
  B.n_coarse = (int)co.size();
  if (B.n_ent > kMaxEnt) return "too many neighbour entries";
  out.insert(out.end(), co.begin(), co.end());
  out.insert(out.end(), sa.begin(), sa.end());
  out.insert(out.end(), fi.begin(), fi.end());
  return nullptr;
}

// Neighbour entries of every leaf; fails with MRB_E_TOPOLOGY if the forest is not
// graded.  Large forests are split over host threads (read-only lookups), each
// filling its own entry list; the lists are then concatenated in forest order.
mrb_status build_descriptors(mrb_ctx* c) {
  HostTimer ht(&c->hus_desc);
  const int d = c->cfg.dim, jmax = c->cfg.jmax;
  const int n = (int)c->leaves.size();
  std::vector<BlockDesc> hblk(n);
  int nt = 1;
  if (n >= (int)c->desc_thread_min) {
    const int hc = (int)std::max(1u, std::thread::hardware_concurrency());
    nt = std::max(1, std::min({16, hc, n / 64}));
  }
  // per-thread entry lists kept between calls (no fresh pages to fault in)
  if ((int)c->desc_parts.size() < nt) c->desc_parts.resize(nt);
  auto& part = c->desc_parts;
  std::vector<const char*> err(nt, nullptr);
  auto work = [&](int t) {
    const int lo = (int)((long)n * t / nt), hi = (int)((long)n * (t + 1) / nt);
    std::vector<NbEntry> co, sa, fi;
    part[t].clear();
    part[t].reserve((size_t)(hi - lo) * (d == 2 ? 13 : 57));
    for (int i = lo; i < hi && !err[t]; ++i) err[t] = block_entries(c, i, part[t], hblk[i], co, sa, fi);
  };
  {
    HostTimer hp(&c->hus_desc_par);
    c->pool.run(nt, work);
  }
  for (int t = 0; t < nt; ++t)
    if (err[t]) return fail(c, MRB_E_TOPOLOGY, err[t]);
  std::vector<NbEntry>& hnb = c->hnb_next;
  hnb.clear();
  size_t total = 0;
  for (int t = 0; t < nt; ++t) total += part[t].size();
  hnb.reserve(total);
  for (int t = 0; t < nt; ++t) {
    const int lo = (int)((long)n * t / nt), hi = (int)((long)n * (t + 1) / nt);
    const int off = (int)hnb.size();
    for (int i = lo; i < hi; ++i) hblk[i].nb_begin += off;
    hnb.insert(hnb.end(), part[t].begin(), part[t].end());
  }
  // blocks grouped by level (plain form launches one sweep per level)
  std::vector<int> level_off(jmax + 2, 0), hlist(n, 0);
  for (auto& L : c->leaves) level_off[L.level + 1]++;
  for (int l = 1; l <= jmax + 1; ++l) level_off[l] += level_off[l - 1];
  std::vector<int> fill(level_off.begin(), level_off.end());
  for (int i = 0; i < n; ++i) hlist[fill[c->leaves[i].level]++] = i;
  c->hblk.swap(hblk);
  c->hnb.swap(hnb);
  c->level_off.swap(level_off);
  c->hlist.swap(hlist);
  return MRB_OK;
}

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// One host->device copy of the packed topology: header, current blocks and
// entries, the level-sorted block list, and optionally the refinement parents
// (with their entries) or the coarsening families.
mrb_status upload_topo(mrb_ctx* c, const std::vector<BlockDesc>* pblk = nullptr,
                       const std::vector<NbEntry>* pnb = nullptr, const std::vector<RefineDesc>* ref = nullptr,
                       const std::vector<FamilyDesc>* fam = nullptr, const std::vector<int>* smap = nullptr) {
  HostTimer ht(&c->hus_upload);
  TopoHeader h;
  std::memset(&h, 0, sizeof h);
  h.n_blocks = (int)c->hblk.size();
  h.n_ref = ref ? (int)ref->size() : 0;
  h.n_fam = fam ? (int)fam->size() : 0;
  h.n_pblk = pblk ? (int)pblk->size() : 0;
  // entries padded to the largest count, block b's at b * stride
  auto stride_of = [](const std::vector<BlockDesc>& v) {
    int m = 1;
    for (const BlockDesc& d : v) m = std::max(m, d.n_ent);
    return m;
  };
  h.nb_stride = stride_of(c->hblk);
  h.pnb_stride = pblk ? stride_of(*pblk) : 1;
  size_t off = align16(sizeof(TopoHeader));
  auto place = [&](size_t bytes) {
    size_t o = off;
    off = align16(off + bytes);
    return (int)o;
  };
  h.off_blk = place(c->hblk.size() * sizeof(BlockDesc));
  h.off_nb = place(c->hblk.size() * (size_t)h.nb_stride * sizeof(NbEntry));
  h.off_list = place(c->hlist.size() * sizeof(int));
  h.off_pblk = place(pblk ? pblk->size() * sizeof(BlockDesc) : 0);
  h.off_pnb = place(pblk ? pblk->size() * (size_t)h.pnb_stride * sizeof(NbEntry) : 0);
  h.off_ref = place(ref ? ref->size() * sizeof(RefineDesc) : 0);
  h.off_fam = place(fam ? fam->size() * sizeof(FamilyDesc) : 0);
  h.off_smap = smap ? place(smap->size() * sizeof(int)) : 0;
  const size_t total = off;
  if (total > (size_t)0x7fffffff) return fail(c, MRB_E_CAPACITY, "topology buffer exceeds 2 GiB");
  if (total > c->arena_cap) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->work_arena) HIPCHK(c, hipFree(c->work_arena));
    c->work_arena = nullptr;
    const size_t cap = total + total / 2 + 4096;
    HIPCHK(c, hipMalloc((void**)&c->work_arena, cap));
    c->arena_cap = cap;
  }
  c->arena = c->work_arena;
  c->arena_hdr = h;
  c->arena_bytes = total;
  Staging& S = c->st_topo[c->st_cur];
  c->st_cur ^= 1;
  if (S.pending) {
    HIPCHK(c, hipEventSynchronize(S.ev));
    S.pending = false;
  }
  if (!S.ev) HIPCHK(c, hipEventCreateWithFlags(&S.ev, hipEventDisableTiming));
  if (total > S.cap) {
    if (S.h) HIPCHK(c, hipHostFree(S.h));
    S.h = nullptr;
    const size_t cap = total + total / 2 + 4096;
    HIPCHK(c, hipHostMalloc(&S.h, cap, hipHostMallocDefault));
    S.cap = cap;
  }
  char* b = (char*)S.h;
  std::memcpy(b, &h, sizeof h);
  auto put = [&](int o, const void* p, size_t n) { if (n) std::memcpy(b + o, p, n); };
  put(h.off_blk, c->hblk.data(), c->hblk.size() * sizeof(BlockDesc));
  auto put_entries = [&](int o, int stride, const std::vector<BlockDesc>& v, const std::vector<NbEntry>& e) {
    for (size_t i = 0; i < v.size(); ++i)
      put(o + (int)(i * stride * sizeof(NbEntry)), e.data() + v[i].nb_begin, v[i].n_ent * sizeof(NbEntry));
  };
  put_entries(h.off_nb, h.nb_stride, c->hblk, c->hnb);
  put(h.off_list, c->hlist.data(), c->hlist.size() * sizeof(int));
  if (pblk) put(h.off_pblk, pblk->data(), pblk->size() * sizeof(BlockDesc));
  if (pblk && pnb) put_entries(h.off_pnb, h.pnb_stride, *pblk, *pnb);
  if (ref) put(h.off_ref, ref->data(), ref->size() * sizeof(RefineDesc));
  if (fam) put(h.off_fam, fam->data(), fam->size() * sizeof(FamilyDesc));
  if (smap) put(h.off_smap, smap->data(), smap->size() * sizeof(int));
  HIPCHK(c, hipMemcpyAsync(c->arena, S.h, total, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipEventRecord(S.ev, c->stream));
  S.pending = true;
  return MRB_OK;
}

Topo topo(const mrb_ctx* c) { return Topo{c->arena, c->arena_hdr}; }

// ---- memo of topology transitions (small forests) ----------------------------------
constexpr size_t kMemoMaxLeaves = 1024;
constexpr size_t kMemoEntries = 8;

// everything a refine-all (kind 0), a coarsening (kind 1) or a marked refinement
// (kind 2) plan depends on: the leaves with their slots, the free-list tail the plan
// can consume, and the flags or the mask
void memo_material(const mrb_ctx* c, int kind, const int8_t* flags, std::vector<int>& m) {
  const size_t n = c->leaves.size(), nch = (size_t)1 << c->cfg.dim;
  m.clear();
  m.reserve(n * 6 + 8);
  m.push_back(kind);
  m.push_back((int)n);
  for (const Leaf& L : c->leaves) {
    m.push_back(L.level);
    m.push_back(L.c[0]);
    m.push_back(L.c[1]);
    m.push_back(L.c[2]);
    m.push_back(L.slot);
  }
  const size_t k = std::min(c->free_slots.size(), kind == 1 ? n / nch + 1 : n * nch);
  m.push_back((int)c->free_slots.size());
  m.insert(m.end(), c->free_slots.end() - (long)k, c->free_slots.end());
  if (kind >= 1)   // coarsening: the flags; marked refinement: the mask
    for (size_t i = 0; i < n; ++i) m.push_back(flags[i]);
}

mrb_ctx::Memo* memo_find(mrb_ctx* c, int kind, const std::vector<int>& m) {
  for (auto& e : c->memo)
    if (e.kind == kind && e.material == m) return &e;
  return nullptr;
}

void memo_apply(mrb_ctx* c, mrb_ctx::Memo& e) {
  c->leaves = e.leaves;
  c->index.clear();
  for (size_t i = 0; i < c->leaves.size(); ++i) c->index.set(pack_key(c->leaves[i].level, c->leaves[i].c), (int)i);
  c->hblk = e.hblk;
  c->hnb = e.hnb;
  c->hlist = e.hlist;
  c->level_off = e.level_off;
  c->free_slots.resize(c->free_slots.size() - e.pop);
  c->free_slots.insert(c->free_slots.end(), e.pushed.begin(), e.pushed.end());
  c->arena = e.arena;
  c->arena_hdr = e.hdr;
  c->arena_bytes = e.arena_bytes;
  e.last_use = ++c->memo_clock;
  ++c->memo_hits;
}

// Remember the transition just planned and uploaded (the current state is its result).
mrb_status memo_record(mrb_ctx* c, int kind, std::vector<int>& material, size_t pop, const std::vector<int>& pushed,
                       int pending_ref, int nfam, int npar) {
  if (material.empty() || c->leaves.size() > kMemoMaxLeaves) return MRB_OK;
  mrb_ctx::Memo* e = nullptr;
  if (c->memo.size() < kMemoEntries) {
    c->memo.emplace_back();
    e = &c->memo.back();
  } else {
    e = &c->memo[0];
    for (auto& x : c->memo)
      if (x.last_use < e->last_use) e = &x;
  }
  if (e->arena && e->arena_bytes < c->arena_bytes) {
    HIPCHK(c, hipStreamSynchronize(c->stream));  // queued kernels may still read it
    HIPCHK(c, hipFree(e->arena));
    e->arena = nullptr;
  }
  if (!e->arena) HIPCHK(c, hipMalloc((void**)&e->arena, c->arena_bytes));
  e->arena_bytes = c->arena_bytes;
  e->hdr = c->arena_hdr;
  e->kind = kind;
  e->material.swap(material);
  e->last_use = ++c->memo_clock;
  e->leaves = c->leaves;
  e->hblk = c->hblk;
  e->hnb = c->hnb;
  e->hlist = c->hlist;
  e->level_off = c->level_off;
  e->pop = pop;
  e->pushed = pushed;
  e->pending_ref = pending_ref;
  e->nfam = nfam;
  e->npar = npar;
  e->smap = e->hdr.off_smap ? (const int*)(e->arena + e->hdr.off_smap) : nullptr;
  HIPCHK(c, hipMemcpyAsync(e->arena, c->arena, c->arena_bytes, hipMemcpyDeviceToDevice, c->stream));
  return MRB_OK;
}

int grid_for(const mrb_ctx* c, long n) { return (int)std::max(1L, std::min((long)c->grid, n)); }

// blocks of the current grid (the device's count while it holds the topology)
size_t nblk(const mrb_ctx* c) { return c->dev.active ? (size_t)c->dev.n : c->hblk.size(); }

mrb_status check_forest(mrb_ctx* c) {
  const int d = c->cfg.dim, jmax = c->cfg.jmax;
  // no duplicates, no leaf inside another, volumes sum to the domain
  unsigned __int128 vol = 0, total = (unsigned __int128)1 << (d * jmax);
  for (auto& L : c->leaves) {
    vol += (unsigned __int128)1 << (d * (jmax - L.level));
    int pc[3] = {L.c[0], L.c[1], L.c[2]};
    for (int l = L.level - 1; l >= 1; --l) {
      for (int a = 0; a < d; ++a) pc[a] >>= 1;
      if (c->index.find(pack_key(l, pc)) >= 0) return fail(c, MRB_E_TOPOLOGY, "blocks overlap");
    }
  }
  if (vol != total) return fail(c, MRB_E_TOPOLOGY, "forest does not tile the domain");
  return MRB_OK;
}

// Algorithmic HBM bytes per interior node and field of RK stage s: stage 1 reads
// u and writes k1; stages 2-3 read u and k_{s-1} and write k_s; stage 4 reads u,
// k3, k1, k2 and writes u_new (FP64: 16+24+24+40 = 104; mixed: 12+16+16+28 = 72).
double stage_bytes(const mrb_ctx* c, int s) {
  const double kb = c->cfg.precision == MRB_MIXED ? 4.0 : 8.0;
  switch (s) {
    case 1: return 8.0 + kb;
    case 2: case 3: return 8.0 + 2.0 * kb;
    default: return 8.0 + 3.0 * kb + 8.0;
  }
}

// sub-tiles per axis for the fused stage: the tuned choice, else the smallest
// count whose workgroups cover the chip twice
int pick_nsub(const mrb_ctx* c) {
  int v[8];
  const int nv = stage_variants(c->shape, c->cfg.precision, v, 8);
  if (nv == 0) return 0;
  if (c->nsub) {
    for (int i = 0; i < nv; ++i)
      if (v[i] == c->nsub) return c->nsub;
  }
  std::sort(v, v + nv);
  const long n = (long)nblk(c);
  for (int i = 0; i < nv; ++i) {
    long w = n;
    for (int a = 0; a < c->cfg.dim; ++a) w *= v[i];
    if (w >= 2L * c->ncu) return v[i];
  }
  return v[nv - 1];
}

// threads per workgroup of the stage kernel: the tuned choice for the tuned tiling
int pick_tpb(const mrb_ctx* c, int nsub) { return c->nsub == nsub ? c->tpb : 256; }

// threads per workgroup of the analysis kernel: the tuned choice for whole blocks
int mr_tpb(const mrb_ctx* c, int nsub) { return nsub == 1 ? c->tpb_mr : 256; }

// sub-tiles per axis for the analysis / refinement kernels: the smallest count whose
// workgroups (n_items each) cover the chip twice
int pick_aux(const mrb_ctx* c, long n_items, int forced = 0) {
  int v[8];
  const int nv = aux_variants(c->shape, 0, v, 8);
  for (int i = 0; i < nv; ++i)
    if (forced && v[i] == forced) return forced;
  if (forced < 0) return 1;  // whole blocks
  std::sort(v, v + nv);
  for (int i = 0; i < nv; ++i) {
    long w = n_items;
    for (int a = 0; a < c->cfg.dim; ++a) w *= v[i];
    if (w >= 2L * c->ncu) return v[i];
  }
  return v[nv - 1];
}

// launch one RK stage (fused) or ghost + RHS per level (plain)
mrb_status run_stage(mrb_ctx* c, int s, const StageArgs& a0, bool fixed_grid = false, bool time_it = true) {
  StageArgs a = a0;
  const int n = (int)nblk(c);
  if (c->cfg.form == MRB_FORM_PLAIN) {
    for (int l = 1; l <= c->cfg.jmax; ++l) {
      const int b0 = c->level_off[l], b1 = c->level_off[l + 1];
      if (b1 == b0) continue;
      a.lvl_begin = b0;
      a.lvl_end = b1;
      TimeScope ts(c, T_RHS_PLAIN, (double)(b1 - b0) * c->bsz * stage_bytes(c, s));
      HIPCHK(c, launch_plain(c->shape, grid_for(c, b1 - b0), a, c->stream));
    }
    return MRB_OK;
  }
  const int nsub = pick_nsub(c);
  long work = n;
  for (int d = 0; d < c->cfg.dim; ++d) work *= nsub;
  TimeScope ts(c, T_STAGE, (double)n * c->bsz * stage_bytes(c, s), 1, time_it);
  HIPCHK(c, launch_stage(c->shape, c->cfg.precision, Variant{nsub, pick_tpb(c, nsub)},
                         fixed_grid ? c->grid : grid_for(c, work), a,
                         c->stream));
  return MRB_OK;
}

StageArgs stage_args(mrb_ctx* c) {
  StageArgs a;
  std::memset(&a, 0, sizeof a);
  a.topo = topo(c);
  a.lvl_begin = 0;
  a.lvl_end = -1;
  a.order = c->dev.active ? 0 : c->order;   // the device path builds no level-sorted list
  a.u = c->u;
  a.unew = c->unew;
  a.k1 = c->k[0];
  a.k2 = c->k[1];
  a.k3 = c->k[2];
  for (int f = 0; f < 4; ++f) a.off[f] = f < (int)c->off.size() ? c->off[f] : 0.0;
  a.lt = c->lt;
  a.ph = c->ph;
  a.ghost = c->dghost;
  return a;
}

bool sweep_in_one(const mrb_ctx* c) {
  return c->cfg.form == MRB_FORM_FUSED && (c->sweep_mode == 1 || (c->sweep_mode == 2 && c->sweep_one_tuned));
}

// every leaf on one level (the overlapped-tile RK4 step's condition)
bool one_level(const mrb_ctx* c) {
  const long n = (long)nblk(c);
  if (n == 0) return false;
  if (c->dev.active) {
    for (int l = 0; l < kMaxLevels; ++l)
      if (c->dev.hist[l] == n) return true;
    return false;
  }
  for (size_t l = 0; l + 1 < c->level_off.size(); ++l)
    if (c->level_off[l + 1] - c->level_off[l] == n) return true;
  return false;
}

// sub-tiles per axis of the overlapped-tile RK4 step, or 0 where it does not apply
int rk4t_pick(const mrb_ctx* c) {
  if (c->cfg.form != MRB_FORM_FUSED) return 0;
  if (!(c->sweep_mode == 3 || (c->sweep_mode == 2 && c->rk4t_tuned))) return 0;
  int v[8];
  const int nv = rk4t_variants(c->shape, c->cfg.precision, v, 8);
  if (nv == 0 || !one_level(c)) return 0;
  for (int i = 0; i < nv; ++i)
    if (v[i] == c->rk4t_nsub) return v[i];
  return v[0];
}

// arguments of the overlapped-tile RK4 step (stage coefficients as in sweep)
Rk4tArgs rk4t_args(mrb_ctx* c, double t, double dt) {
  const double h2 = dt * 0.5;
  const double ts[4] = {t, t + h2, t + h2, t + dt};
  const double alpha[4] = {0.0, h2, h2, dt};
  Rk4tArgs ra;
  std::memset(&ra, 0, sizeof ra);
  ra.topo = topo(c);
  ra.u = c->u;
  ra.unew = c->unew;
  ra.h6 = dt / 6.0;
  ra.off = c->off.empty() ? 0.0 : c->off[0];
  ra.lt = c->lt;
  ra.ph = c->ph;
  for (int s = 0; s < 4; ++s) {
    ra.alpha[s] = alpha[s];
    ra.cfac[s] = 1.0;
    if (c->cfg.physics == MRB_ADV_SWIRL && c->cfg.phys[0] > 0.0) ra.cfac[s] = std::cos(M_PI * ts[s] / c->cfg.phys[0]);
  }
  return ra;
}

// launch the overlapped-tile RK4 step (tn sub-tiles per axis), with the analysis of
// u_new folded in or not
mrb_status launch_tiled(mrb_ctx* c, int tn, const Rk4tArgs& ra, bool analysis, int tpb = 256, bool refine = false,
                        bool mothers = false) {
  const long work = (long)nblk(c) * tn * tn;
  // algorithmic bytes of the work the launch performs, counted as for the stage,
  // analysis and refinement launches it replaces (an RK4 step: the four stages' bytes
  // per node; the analysis: 8 per node; the refinement: 8 (1 + 2^d) per parent node).
  // The launch itself reads u (or the parents' u) once and writes u_new once.
  double per_node = 0.0;
  for (int s = 1; s <= 4; ++s) per_node += stage_bytes(c, s);
  if (analysis) per_node += 8.0;
  const double n = (double)nblk(c), nch = (double)(1 << c->cfg.dim);
  double bytes = n * c->bsz * per_node + (refine ? n / nch * c->bsz * 8.0 * (1.0 + nch) : 0.0);
  if (mothers) bytes += n / nch * c->bsz * 8.0;   // the second analysis, on the mothers
  if (analysis) {
    // sub-tiles leave partial maxima for the host (the launch's flag bank)
    if (tn > 1 && !ra.part) return fail(c, MRB_E_STATE, "tile analysis: no partial-maximum buffer");
    c->part_st.parts = tn > 1 ? tn * tn : 0;
    c->part_st.n = (int)nblk(c);
    c->part_st.level = c->leaves.empty() ? 0 : c->leaves[0].level;
  }
  TimeScope rs(c, T_RK4T, bytes);
  HIPCHK(c, launch_rk4t(c->shape, c->cfg.precision, tn, analysis, refine, mothers, tpb, grid_for(c, work), ra,
                        c->stream));
  return MRB_OK;
}

// the analysis outputs of a folded first pass (flag set 0; no speculated mothers)
void rk4t_analysis_args(mrb_ctx* c, Rk4tArgs& ra, const int* smap) {
  ra.flags = c->dflags;
  ra.maxd = c->dmaxd;
  ra.part = c->dpart;
  ra.thr = c->thr.empty() ? 0.0 : c->thr[0];
  ra.smap = smap;
}

// the four stages of one RK4 step; results go to k1..k3 and u_new (u is read only).
// fixed_grid (graph capture) always takes the four-launch path.
mrb_status sweep(mrb_ctx* c, double t, double dt, bool fixed_grid = false) {
  const double h2 = dt * 0.5, h6 = dt / 6.0;
  const double ts[4] = {t, t + h2, t + h2, t + dt};
  StageArgs a = stage_args(c);
  a.h6 = h6;
  const double alpha[4] = {0.0, h2, h2, dt};
  const int tn = fixed_grid ? 0 : rk4t_pick(c);
  if (tn > 0) return launch_tiled(c, tn, rk4t_args(c, t, dt), false);
  // fused form: one event pair around the four stage launches
  const bool fused = c->cfg.form == MRB_FORM_FUSED;
  double sweep_bytes = 0.0;
  for (int s = 1; s <= 4; ++s) sweep_bytes += (double)nblk(c) * c->bsz * stage_bytes(c, s);
  TimeScope sweep_scope(c, T_STAGE, sweep_bytes, 4, fused);
  if (!fixed_grid && sweep_in_one(c)) {
    SweepArgs sa;
    std::memset(&sa, 0, sizeof sa);
    sa.a = a;
    for (int s = 0; s < 4; ++s) {
      sa.alpha[s] = alpha[s];
      sa.cfac[s] = 1.0;
      if (c->cfg.physics == MRB_ADV_SWIRL && c->cfg.phys[0] > 0.0) sa.cfac[s] = std::cos(M_PI * ts[s] / c->cfg.phys[0]);
    }
    sa.bar = c->dbar;
    sa.err = c->d_err;
    sa.spin = 1u << 22;
    const int nsub = pick_nsub(c);
    long work = (long)nblk(c);
    for (int d = 0; d < c->cfg.dim; ++d) work *= nsub;
    HIPCHK(c, launch_sweep(c->shape, c->cfg.precision, Variant{nsub}, (int)std::min(work, 1L << 30), sa, c->stream,
                           &c->sweep_grid));
    return MRB_OK;
  }
  for (int s = 1; s <= 4; ++s) {
    a.stage = s;
    a.alpha = alpha[s - 1];
    a.kprev = s > 1 ? c->k[s - 2] : nullptr;
    a.kout = s < 4 ? c->k[s - 1] : nullptr;
    a.cfac = 1.0;
    if (c->cfg.physics == MRB_ADV_SWIRL && c->cfg.phys[0] > 0.0) a.cfac = std::cos(M_PI * ts[s - 1] / c->cfg.phys[0]);
    mrb_status r = run_stage(c, s, a, fixed_grid, !fused);
    if (r) return r;
  }
  return MRB_OK;
}

// the shock-capturing filter after a time step (Navier-Stokes with r_th = phys[3] > 0)
bool filter_on(const mrb_ctx* c) { return c->cfg.physics == MRB_NS2D && c->cfg.phys[3] > 0.0; }

mrb_status do_filter(mrb_ctx* c) {
  const long n = (long)nblk(c);
  FilterArgs a{topo(c), c->u, c->unew, c->cfg.phys[3]};
  {
    TimeScope ts(c, T_FILTER, (double)n * c->bsz * 16.0);
    HIPCHK(c, launch_filter(c->shape, grid_for(c, n), a, c->stream));
  }
  std::swap(c->u, c->unew);
  return MRB_OK;
}

mrb_status do_rk4(mrb_ctx* c, double t, double dt) {
  mrb_status r = sweep(c, t, dt);
  if (r) return r;
  std::swap(c->u, c->unew);
  if (filter_on(c) && (r = do_filter(c))) return r;
  c->n_rk4++;
  c->n_block_updates += (long)nblk(c);
  return MRB_OK;
}

mrb_status do_adapt(mrb_ctx* c, int* npass, bool first_launched = false, bool first_fused = false,
                    bool second_folded = false, bool first_tiled = false);
mrb_ctx::Memo* spec_entry(mrb_ctx* c);

// the speculated coarsening of the current grid merges every block (and writes its
// mothers in the first analysis pass)
bool spec_all_merge(mrb_ctx* c) {
  mrb_ctx::Memo* e = spec_entry(c);
  return e && e->smap && c->dmq && (long)e->nfam * (1 << c->cfg.dim) == (long)nblk(c);
}

// The RK4 step and the first analysis pass of its adapt as one overlapped-tile launch,
// where the forest is on one level and that form is selected (else *done = false and
// nothing is launched); then the rest of the adapt.
mrb_status rk4_adapt_tiled(mrb_ctx* c, double t, double dt, bool* done, bool refine) {
  *done = false;
  int tn = rk4t_pick(c), tpb = 256;
  if (tn == 0 || filter_on(c) || c->ana_nsub < 0) return MRB_OK;
  if (refine && (long)c->pending_ref * (1 << c->cfg.dim) != (long)nblk(c))
    return fail(c, MRB_E_STATE, "folded refinement: not every block was refined");
  if (refine && c->ma_nsub > 0 && spec_all_merge(c)) {
    tn = c->ma_nsub;
    tpb = c->ma_tpb;
  } else if (refine && c->ref_nsub > 0) {
    tn = c->ref_nsub;
    tpb = c->ref_tpb;
  } else if (c->ana_nsub > 0) {
    tn = c->ana_nsub;
    tpb = c->ana_tpb;
  }
  mrb_ctx::Memo* e = spec_entry(c);
  const bool fused = e && e->smap;
  // the speculated coarsening merges every block (the mothers are on one level again):
  // its second analysis can be folded in too
  const bool mothers = refine && spec_all_merge(c);
  Rk4tArgs ra = rk4t_args(c, t, dt);
  c->flag_set = 0;
  rk4t_analysis_args(c, ra, fused ? e->smap : nullptr);
  ra.mq = mothers ? c->dmq : nullptr;
  c->mq_parts = tn * tn;
  mrb_status r = launch_tiled(c, tn, ra, true, tpb, refine, mothers);
  if (r) return r;
  std::swap(c->u, c->unew);
  c->n_rk4++;
  c->n_block_updates += (long)nblk(c);
  *done = true;
  return do_adapt(c, nullptr, true, fused, mothers, true);
}

// the step's refinement can be folded into the tile launch: the forest is on one level
// below jmax (refine-all refines every block, the children are on one level) and the
// tile step with the first analysis folded in is selected for them
bool refine_foldable(const mrb_ctx* c) {
  if (c->cfg.form != MRB_FORM_FUSED || c->cfg.dim != 2 || filter_on(c) || c->ana_nsub < 0 || !c->ref_fold)
    return false;
  if (!(c->sweep_mode == 3 || (c->sweep_mode == 2 && c->rk4t_tuned))) return false;
  int v[8];
  if (rk4t_variants(c->shape, c->cfg.precision, v, 8) == 0 || !one_level(c)) return false;
  return !c->leaves.empty() && c->leaves[0].level < c->cfg.jmax && !c->dev.active;
}

// refinement kernel over the uploaded plan (nref parents); fixed_grid for graph capture
mrb_status launch_refine_kernel(mrb_ctx* c, int nref, bool fixed_grid) {
  const int nch = 1 << c->cfg.dim;
  RefineArgs a{topo(c), c->u};
  const int ns = pick_aux(c, (long)nref * nch, c->nsub_ref);
  long work = (long)nref * nch;
  for (int q = 0; q < c->cfg.dim; ++q) work *= ns;
  TimeScope ts(c, T_REFINE, (double)nref * c->bsz * 8.0 * (1 + nch));
  HIPCHK(c, launch_refine(c->shape, ns, fixed_grid ? c->grid : grid_for(c, work), a, c->stream));
  return MRB_OK;
}

// Plan the safety-zone refinement (new forest, descriptors, one upload) and, if
// launch is set, run the refinement kernel.
mrb_status do_refine(mrb_ctx* c, const std::vector<int>& par, bool launch, bool memoize = false,
                     const int8_t* mask = nullptr);

mrb_status do_refine_all(mrb_ctx* c, bool launch = true) {
  std::vector<int> par;
  for (int i = 0; i < (int)c->leaves.size(); ++i)
    if (c->leaves[i].level < c->cfg.jmax) par.push_back(i);
  return do_refine(c, par, launch, true);
}

// refine the listed blocks (forest positions, all below jmax; the caller keeps the
// grid graded)
mrb_status do_refine(mrb_ctx* c, const std::vector<int>& par, bool launch, bool memoize, const int8_t* mask) {
  HostTimer ht(&c->hus_refine_plan);
  const int d = c->cfg.dim, nch = 1 << d;
  c->pending_ref = 0;
  if (par.empty()) {
    // the upload still clears the previous refinement plan of the header
    return c->hcount_ref_zero ? MRB_OK : (c->hcount_ref_zero = true, upload_topo(c));
  }
  std::vector<int> material;
  if (memoize && c->leaves.size() <= kMemoMaxLeaves) {
    memo_material(c, mask ? 2 : 0, mask, material);
    if (mrb_ctx::Memo* e = memo_find(c, mask ? 2 : 0, material)) {
      memo_apply(c, *e);
      c->hcount_ref_zero = false;
      c->n_refined += e->npar;
      c->have_flags = false;
      c->pending_ref = e->pending_ref;
      if (!launch) return MRB_OK;
      return launch_refine_kernel(c, c->pending_ref, false);
    }
  }
  c->hcount_ref_zero = false;
  if (c->free_slots.size() < par.size() * nch) return fail(c, MRB_E_CAPACITY, "refine_all: pool too small");
  // parents' descriptors and entries on the grid before refinement
  std::vector<BlockDesc> pblk(par.size());
  std::vector<NbEntry> pnb;
  std::vector<RefineDesc> ref(par.size());
  std::vector<Leaf> kids;
  kids.reserve(par.size() * nch);
  std::vector<int> taken;
  for (size_t r = 0; r < par.size(); ++r) {
    const Leaf& P = c->leaves[par[r]];
    pblk[r] = c->hblk[par[r]];
    pblk[r].nb_begin = (int)pnb.size();
    pnb.insert(pnb.end(), c->hnb.begin() + c->hblk[par[r]].nb_begin,
               c->hnb.begin() + c->hblk[par[r]].nb_begin + c->hblk[par[r]].n_ent);
    for (int b = 0; b < 8; ++b) ref[r].child[b] = -1;
    for (int b = 0; b < nch; ++b) {
      const int slot = c->free_slots.back();
      c->free_slots.pop_back();
      taken.push_back(slot);
      ref[r].child[b] = slot;
      Leaf K;
      K.level = P.level + 1;
      K.c[0] = K.c[1] = K.c[2] = 0;
      for (int a = 0; a < d; ++a) K.c[a] = 2 * P.c[a] + ((b >> a) & 1);
      K.slot = slot;
      kids.push_back(K);
    }
  }
  // new forest: refined parents leave, children join; parent slots return to the pool
  std::vector<Leaf> old = c->leaves;
  std::vector<char> gone(c->leaves.size(), 0);
  for (int i : par) gone[i] = 1;
  std::vector<Leaf> nl;
  nl.reserve(c->leaves.size() - par.size() + kids.size());
  std::vector<int> freed;
  for (size_t i = 0; i < c->leaves.size(); ++i) {
    if (gone[i]) freed.push_back(c->leaves[i].slot);
    else nl.push_back(c->leaves[i]);
  }
  nl.insert(nl.end(), kids.begin(), kids.end());
  c->leaves.swap(nl);
  sort_and_index(c);
  mrb_status s = build_descriptors(c);
  if (!s) s = upload_topo(c, &pblk, &pnb, &ref, nullptr);
  if (s) {  // internal failure: restore the previous forest
    c->leaves.swap(old);
    sort_and_index(c);
    for (int sl : taken) c->free_slots.push_back(sl);
    build_descriptors(c);
    return s;
  }
  for (int sl : freed) c->free_slots.push_back(sl);
  c->n_refined += (long)par.size();
  c->have_flags = false;
  c->pending_ref = (int)ref.size();
  if (!material.empty() &&
      (s = memo_record(c, mask ? 2 : 0, material, taken.size(), freed, c->pending_ref, 0, (int)par.size())))
    return s;
  if (!launch) return MRB_OK;
  return launch_refine_kernel(c, c->pending_ref, false);
}

MrArgs mr_args(mrb_ctx* c) {
  MrArgs a;
  a.topo = topo(c);
  a.u = c->u;
  a.flags = c->flag_set ? c->dflags2 : c->dflags;
  a.maxd = c->flag_set ? c->dmaxd2 : c->dmaxd;
  a.acc = c->dacc;
  a.done = c->ddone;
  for (int f = 0; f < 4; ++f) a.thr[f] = f < (int)c->thr.size() ? c->thr[f] : 0.0;
  a.smap = nullptr;
  return a;
}

// `spec`: a memoised coarsening of the current grid whose mothers the pass also writes
mrb_status launch_mr_kernel(mrb_ctx* c, bool fixed_grid, const mrb_ctx::Memo* spec = nullptr) {
  const int n = (int)nblk(c);
  MrArgs a = mr_args(c);
  if (spec) a.smap = spec->smap;
  const int ns = pick_aux(c, n, c->nsub_mr);
  long work = n;
  for (int q = 0; q < c->cfg.dim; ++q) work *= ns;
  TimeScope ts(c, T_MR, (double)n * c->bsz * 8.0);
  HIPCHK(c, launch_mr(c->shape, ns, mr_tpb(c, ns), fixed_grid ? c->grid : grid_for(c, work), a, c->stream));
  return MRB_OK;
}

// after a synchronisation: a whole-sweep launch whose barrier wait timed out voids
// the block data (the sweep ended early, so u_new -- now u -- is incomplete); calls
// that need data fail with MRB_E_STATE until new data is loaded.  The barrier words
// are reset for the next launch.
mrb_status check_barrier(mrb_ctx* c) {
  if (!c->h_err || *c->h_err == 0) return MRB_OK;
  *c->h_err = 0;
  c->have_data = false;
  c->have_flags = false;
  HIPCHK(c, hipMemsetAsync(c->dbar, 0, kBarWords * sizeof(unsigned), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return fail(c, MRB_E_DEVICE, "sweep: a grid barrier wait timed out; the block data is void (load new data)");
}

mrb_status wait_stream(mrb_ctx* c);

mrb_status mr_readback(mrb_ctx* c) {
  const int n = (int)nblk(c);
  if (mrb_status r = wait_stream(c)) return r;
  if (mrb_status r = check_barrier(c)) return r;
  c->last_flags.assign(c->h_flags, c->h_flags + n);
  c->last_maxd.assign(c->h_maxd, c->h_maxd + (size_t)n * c->cfg.nfields);
  c->have_flags = true;
  c->n_mr++;
  for (double v : c->last_maxd)
    if (!std::isfinite(v)) return fail(c, MRB_E_NONFINITE, "detail norm is not finite");
  return MRB_OK;
}

mrb_status do_mr_pass(mrb_ctx* c) {
  mrb_status r = launch_mr_kernel(c, false);
  if (r) return r;
  return mr_readback(c);
}

// largest set of complete, flagged families whose merge keeps the grid graded
std::vector<uint64_t> coarsenable(mrb_ctx* c, const int8_t* flags) {
  HostTimer ht(&c->hus_fixed);
  const int d = c->cfg.dim, nch = 1 << d, bs = c->cfg.bs;
  const int n = (int)c->leaves.size();
  // complete families with every member flagged, each found once from its child 0
  std::vector<uint64_t> key;     // mother keys
  std::vector<int> mem;          // members' forest positions, nch per family
  std::vector<int> fam_of(n, -1);
  for (int i = 0; i < n; ++i) {
    const Leaf& L = c->leaves[i];
    if (L.level < 2 || flags[i] != -1) continue;
    bool child0 = true;
    for (int a = 0; a < d; ++a) child0 = child0 && (L.c[a] & 1) == 0;
    if (!child0) continue;
    int p[3] = {L.c[0] >> 1, L.c[1] >> 1, d > 2 ? L.c[2] >> 1 : 0};
    int m[8];
    bool all = true;
    for (int b = 0; b < nch && all; ++b) {
      int ch[3] = {0, 0, 0};
      for (int a = 0; a < d; ++a) ch[a] = 2 * p[a] + ((b >> a) & 1);
      m[b] = c->index.find(pack_key(L.level, ch));
      if (m[b] < 0 || flags[m[b]] != -1) all = false;
    }
    if (!all) continue;
    for (int b = 0; b < nch; ++b) {
      fam_of[m[b]] = (int)key.size();
      mem.push_back(m[b]);
    }
    key.push_back(pack_key(L.level - 1, p));
  }
  // demote families with a finer neighbour whose own family is not (or no longer) a
  // candidate, until stable; each pass checks every family against the previous set
  // (the greatest fixed point does not depend on the order of demotions)
  const int nf = (int)key.size();
  std::vector<char> alive(nf, 1), demote(nf, 0);
  auto check = [&](int f) {
    demote[f] = 0;
    if (!alive[f]) return;
    for (int b = 0; b < nch; ++b) {
      const int mi = mem[(size_t)f * nch + b];
      const Leaf& M = c->leaves[mi];
      const BlockDesc& B = c->hblk[mi];
      for (int e = B.nb_begin; e < B.nb_begin + B.n_ent; ++e) {
        const NbEntry& E = c->hnb[e];
        if (E.dl <= 0) continue;
        int fine[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) fine[a] = wrapi(2 * M.c[a] + (E.o[a] * 2) / (bs - 1), 1 << (M.level + 1));
        const int j = c->index.find(pack_key(M.level + 1, fine));
        if (j < 0 || fam_of[j] < 0 || !alive[fam_of[j]]) {
          demote[f] = 1;
          return;
        }
      }
    }
  };
  const int nt = nf >= 512 ? std::min(8, nf / 256) : 1;
  for (bool changed = true; changed;) {
    c->pool.run(nt, [&](int t) {
      const int lo = (int)((long)nf * t / nt), hi = (int)((long)nf * (t + 1) / nt);
      for (int f = lo; f < hi; ++f) check(f);
    });
    changed = false;
    for (int f = 0; f < nf; ++f)
      if (demote[f]) {
        alive[f] = 0;
        changed = true;
      }
  }
  std::vector<uint64_t> out;
  for (int f = 0; f < nf; ++f)
    if (alive[f]) out.push_back(key[f]);
  std::sort(out.begin(), out.end());
  return out;
}

// a memoised coarsening: adopt its forest and plan, launch the coarsening kernel
// `written`: the analysis pass already wrote the mothers
mrb_status coarsen_from_memo(mrb_ctx* c, mrb_ctx::Memo& e, bool written = false) {
  memo_apply(c, e);
  c->hcount_ref_zero = true;
  CoarsenArgs a{topo(c), c->u};
  const long total = (long)e.nfam * c->np;
  if (!written) {
    TimeScope ts(c, T_COARSEN, (double)total * c->cfg.nfields * 16.0);
    HIPCHK(c, launch_coarsen(c->shape, (int)std::min(4096L, (total + 255) / 256), a, c->stream));
  }
  c->n_fam += e.nfam;
  c->have_flags = false;
  return MRB_OK;
}

mrb_status do_coarsen(mrb_ctx* c, const int8_t* flags, int* ncoarse) {
  HostTimer ht(&c->hus_coarsen_plan);
  const int d = c->cfg.dim, nch = 1 << d;
  std::vector<int> material;
  if (c->leaves.size() <= kMemoMaxLeaves) {
    memo_material(c, 1, flags, material);
    if (mrb_ctx::Memo* e = memo_find(c, 1, material)) {
      if (ncoarse) *ncoarse = e->nfam;
      if (e->nfam == 0) {  // nothing merges: the state stays as it is
        e->last_use = ++c->memo_clock;
        ++c->memo_hits;
        return MRB_OK;
      }
      return coarsen_from_memo(c, *e);
    }
  }
  std::vector<uint64_t> fams = coarsenable(c, flags);
  if (ncoarse) *ncoarse = (int)fams.size();
  if (fams.empty()) {
    if (!material.empty()) {
      // remember that nothing merges here (no device copy needed: state unchanged)
      mrb_status r = memo_record(c, 1, material, 0, std::vector<int>(), 0, 0, 0);
      if (r) return r;
    }
    return MRB_OK;
  }
  if (c->free_slots.size() < fams.size()) return fail(c, MRB_E_CAPACITY, "coarsen: pool too small");
  // Slots: mothers take theirs from the free list in reverse forest order, and the
  // children's slots go back in reverse forest order.  A refinement pushes its
  // parents' slots in forest order and hands out children's slots from the back, so
  // a coarsening that undoes it returns every block to the slot it had: a forest
  // cycling through the same refinement and coarsening repeats its slots exactly and
  // its plans are found in the memo.
  std::vector<int> mslot(fams.size());
  std::vector<std::pair<uint64_t, int>> ord(fams.size());
  for (size_t i = 0; i < fams.size(); ++i) {
    const uint64_t pk = fams[i];
    const int p[3] = {(int)(pk & 0xFFFFF), (int)((pk >> 20) & 0xFFFFF), (int)((pk >> 40) & 0xFFFFF)};
    ord[i] = {morton_of(c, (int)(pk >> 60), p), (int)i};
  }
  std::sort(ord.begin(), ord.end());
  for (size_t k = ord.size(); k-- > 0;) {
    mslot[ord[k].second] = c->free_slots.back();
    c->free_slots.pop_back();
  }
  std::vector<FamilyDesc> fd(fams.size());
  std::vector<char> gone(c->leaves.size(), 0);
  std::vector<int> smap(c->leaves.size(), -1);   // per block: mother slot * 8 + child index
  std::vector<Leaf> parents;
  for (size_t i = 0; i < fams.size(); ++i) {
    const uint64_t pk = fams[i];
    const int l = (int)(pk >> 60);
    int p[3] = {(int)(pk & 0xFFFFF), (int)((pk >> 20) & 0xFFFFF), (int)((pk >> 40) & 0xFFFFF)};
    Leaf P;
    P.level = l;
    for (int a = 0; a < 3; ++a) P.c[a] = p[a];
    P.slot = mslot[i];
    fd[i].parent = P.slot;
    for (int b = 0; b < 8; ++b) fd[i].child[b] = -1;
    for (int b = 0; b < nch; ++b) {
      int ch[3] = {0, 0, 0};
      for (int a = 0; a < d; ++a) ch[a] = 2 * p[a] + ((b >> a) & 1);
      const int mi = c->index.find(pack_key(l + 1, ch));
      fd[i].child[b] = c->leaves[mi].slot;
      gone[mi] = 1;
      smap[mi] = P.slot * 8 + b;
    }
    parents.push_back(P);
  }
  std::vector<Leaf> old = c->leaves;
  std::vector<Leaf> nl;
  std::vector<int> freed;
  for (size_t i = 0; i < c->leaves.size(); ++i) {
    if (gone[i]) freed.push_back(c->leaves[i].slot);
    else nl.push_back(c->leaves[i]);
  }
  std::reverse(freed.begin(), freed.end());
  nl.insert(nl.end(), parents.begin(), parents.end());
  c->leaves.swap(nl);
  sort_and_index(c);
  mrb_status s = build_descriptors(c);
  if (!s) s = upload_topo(c, nullptr, nullptr, nullptr, &fd, material.empty() ? nullptr : &smap);
  if (s) {
    c->leaves.swap(old);
    sort_and_index(c);
    for (const auto& o : ord) c->free_slots.push_back(mslot[o.second]);   // the free list as it was
    build_descriptors(c);
    return s;
  }
  for (int sl : freed) c->free_slots.push_back(sl);
  c->hcount_ref_zero = true;
  if (!material.empty() && (s = memo_record(c, 1, material, fams.size(), freed, 0, (int)fams.size(), 0))) return s;
  CoarsenArgs a{topo(c), c->u};
  const long total = (long)fd.size() * c->np;
  {
    TimeScope ts(c, T_COARSEN, (double)total * c->cfg.nfields * 16.0);
    HIPCHK(c, launch_coarsen(c->shape, (int)std::min(4096L, (total + 255) / 256), a, c->stream));
  }
  c->n_fam += (long)fams.size();
  c->have_flags = false;
  return MRB_OK;
}

// wait for the stream's work so far (the adapt's read-back)
mrb_status wait_stream(mrb_ctx* c) {
  HostTimer ht(&c->hus_wait);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MRB_OK;
}

// flags and maxima of the analysis just finished (mapped set `set`, n blocks)
mrb_status take_flags(mrb_ctx* c, int set, size_t n) {
  if (mrb_status r = check_barrier(c)) return r;
  const int8_t* f = set ? c->h_flags2 : c->h_flags;
  const double* m = set ? c->h_maxd2 : c->h_maxd;
  c->last_flags.assign(f, f + n);
  c->last_maxd.assign(m, m + n * c->cfg.nfields);
  c->have_flags = true;
  c->n_mr++;
  for (double v : c->last_maxd)
    if (!std::isfinite(v)) return fail(c, MRB_E_NONFINITE, "detail norm is not finite");
  return MRB_OK;
}

// Adapt: analysis, coarsening, repeated until nothing merges (Sec. 2.1 item 3).
// On small forests that repeat, the first coarsening is speculated from the memo:
// if the forest is in a state whose first-pass flags were seen last time, the
// memoised coarsening and the second analysis are launched before anything is
// read back; if the first-pass flags then differ, the host state is put back (the
// device data of the uncoarsened grid is untouched: the coarsening writes only new
// slots, and the second analysis writes back into shared nodes the values the first
// one wrote) and the adapt continues from the real flags.
// the memoised coarsening that the last adapt's first-pass flags would give on the
// current grid (the speculation of do_adapt), or null
mrb_ctx::Memo* spec_entry(mrb_ctx* c) {
  const size_t n = c->leaves.size();
  if (n > kMemoMaxLeaves || c->spec_flags.size() != n) return nullptr;
  std::vector<int> mat;
  memo_material(c, 1, c->spec_flags.data(), mat);
  mrb_ctx::Memo* e = memo_find(c, 1, mat);
  return e && e->nfam > 0 ? e : nullptr;
}

// first_launched: the first pass is already queued (graph replay, or folded into the
// overlapped-tile RK4 step); first_fused: that pass was given the speculated
// coarsening's map and wrote its mothers
// The uncoarsened grid's host state, kept while a speculated coarsening is applied
// (put back if the speculation misses).
struct SpecSnap {
  std::vector<Leaf> leaves;
  std::vector<BlockDesc> hblk;
  std::vector<NbEntry> hnb;
  std::vector<int> hlist, level_off, popped;
  size_t npushed = 0, n1 = 0;
  char* arena = nullptr;
  TopoHeader hdr;
  size_t arena_bytes = 0;
  bool ref_zero = false;
  int nfam = 0;
};

// snapshot the grid, then apply the memoised coarsening e (its mothers already written
// when `written`)
mrb_status spec_begin(mrb_ctx* c, mrb_ctx::Memo* e, bool written, SpecSnap& sn) {
  sn.leaves = c->leaves;
  sn.hblk = c->hblk;
  sn.hnb = c->hnb;
  sn.hlist = c->hlist;
  sn.level_off = c->level_off;
  sn.popped.assign(c->free_slots.end() - (long)e->pop, c->free_slots.end());
  sn.npushed = e->pushed.size();
  sn.n1 = c->leaves.size();
  sn.arena = c->arena;
  sn.hdr = c->arena_hdr;
  sn.arena_bytes = c->arena_bytes;
  sn.ref_zero = c->hcount_ref_zero;
  sn.nfam = e->nfam;
  return coarsen_from_memo(c, *e, written);
}

// the first analysis of a tile launch with sub-tiles: each block's maximum over its
// sub-tiles' shares (NaN-propagating, as the analysis kernel's reduction), then the flag
// rule (every block of that launch is on one level), into flag set 0
void ana_combine(mrb_ctx* c) {
  mrb_ctx::PartState& ps = c->part_st;
  if (ps.parts <= 1) return;
  for (int b = 0; b < ps.n; ++b) {
    const double* q = c->h_part + (size_t)b * ps.parts;
    double v = q[0];
    for (int k = 1; k < ps.parts; ++k) {
      const double w = q[k];
      v = v != v ? v : (w != w ? w : (v > w ? v : w));
    }
    c->h_maxd[b] = v;
    c->h_flags[b] = ps.level > 1 && v < c->thr[0] ? (int8_t)-1 : (int8_t)0;
  }
  ps.parts = 0;
}

// the mothers' detail maxima of a folded second analysis: the maximum over their
// children's sub-tile shares (NaN-propagating, as the analysis kernel's reduction), then
// the flag rule, into flag set 1
void mother_flags(mrb_ctx* c) {
  const int nch = 1 << c->cfg.dim, parts = nch * c->mq_parts;
  for (size_t m = 0; m < c->leaves.size(); ++m) {
    double v = c->h_mq[m * parts];
    for (int q = 1; q < parts; ++q) {
      const double w = c->h_mq[m * parts + q];
      v = v != v ? v : (w != w ? w : (v > w ? v : w));
    }
    c->h_maxd2[m] = v;
    c->h_flags2[m] = c->leaves[m].level > 1 && v < c->thr[0] ? (int8_t)-1 : (int8_t)0;
  }
}

// After the wait: keep the speculated coarsening if the first pass's flags are the ones it
// was made from, else put the uncoarsened grid back; then coarsen until nothing merges.
mrb_status spec_finish(mrb_ctx* c, SpecSnap& sn, bool second_folded, int* npass) {
  mrb_status s;
  int passes = 1;
  const size_t n1 = sn.n1;
  if (std::equal(c->h_flags, c->h_flags + n1, c->spec_flags.begin())) {
    ++c->spec_hits;
    if ((s = take_flags(c, 0, n1))) return s;
    if (second_folded) mother_flags(c);
    if ((s = take_flags(c, 1, c->leaves.size()))) return s;
    passes = 2;
  } else {
    ++c->spec_misses;
    c->leaves.swap(sn.leaves);
    c->index.clear();
    for (size_t i = 0; i < c->leaves.size(); ++i) c->index.set(pack_key(c->leaves[i].level, c->leaves[i].c), (int)i);
    c->hblk.swap(sn.hblk);
    c->hnb.swap(sn.hnb);
    c->hlist.swap(sn.hlist);
    c->level_off.swap(sn.level_off);
    c->free_slots.resize(c->free_slots.size() - sn.npushed);
    c->free_slots.insert(c->free_slots.end(), sn.popped.begin(), sn.popped.end());
    c->arena = sn.arena;
    c->arena_hdr = sn.hdr;
    c->arena_bytes = sn.arena_bytes;
    c->hcount_ref_zero = sn.ref_zero;
    c->n_fam -= sn.nfam;
    if ((s = take_flags(c, 0, n1))) return s;
    c->spec_flags = c->last_flags;
  }
  for (;;) {
    int nc = 0;
    std::vector<int8_t> fl = c->last_flags;
    if ((s = do_coarsen(c, fl.data(), &nc))) return s;
    if (nc == 0) break;
    if (passes > c->cfg.jmax + 2) return fail(c, MRB_E_STATE, "adapt did not reach a fixed point");
    if ((s = do_mr_pass(c))) return s;
    ++passes;
  }
  if (npass) *npass = passes;
  return MRB_OK;
}

// first_tiled: the first pass ran inside the tile launch just made (its sub-tiles, if any,
// left partial maxima for ana_combine)
mrb_status do_adapt(mrb_ctx* c, int* npass, bool first_launched, bool first_fused, bool second_folded,
                    bool first_tiled) {
  mrb_status s;
  c->flag_set = 0;
  const size_t n1 = c->leaves.size();
  mrb_ctx::Memo* e = spec_entry(c);
  // a first pass launched here also writes the speculated mothers
  const bool fused = e && e->smap && (first_launched ? first_fused : true);
  if (!first_launched && (s = launch_mr_kernel(c, false, fused ? e : nullptr))) return s;
  if (!e) {
    if ((s = wait_stream(c))) return s;
    if (first_tiled) ana_combine(c);
    if ((s = take_flags(c, 0, n1))) return s;
    c->spec_flags = c->last_flags;
    for (int passes = 1;; ++passes) {
      int nc = 0;
      std::vector<int8_t> fl = c->last_flags;
      if ((s = do_coarsen(c, fl.data(), &nc))) return s;
      if (nc == 0) {
        if (npass) *npass = passes;
        return MRB_OK;
      }
      if (passes > c->cfg.jmax + 2) return fail(c, MRB_E_STATE, "adapt did not reach a fixed point");
      if ((s = do_mr_pass(c))) return s;
    }
  }
  SpecSnap sn;
  if ((s = spec_begin(c, e, fused, sn))) return s;
  if (!second_folded) {
    c->flag_set = 1;
    s = launch_mr_kernel(c, false);
    c->flag_set = 0;
    if (s) return s;
  }
  if ((s = wait_stream(c))) return s;
  if (first_tiled) ana_combine(c);
  return spec_finish(c, sn, second_folded, npass);
}

// ---------------------------------------------------------------------------
// Steps of a forest that cycles through the one-launch step: before each step it is on
// one level below jmax, refine-all, RK4 and both analysis passes run in one tile
// launch, and the speculated coarsening merges every block back into the same forest
// with the same slots.  The next step's launch is then queued before this step's flags
// are read, so the device never waits for the host: the host state after the queued
// step's refinement and speculated coarsening is the same as before, and only the
// data buffers (u and u_new swap each step) and the flag outputs (two banks, alternating)
// differ.  If a step's flags miss the speculation, or its second pass would merge
// more, the queued step is taken back -- it wrote only the other data buffer and free
// slots, so the step's own results are intact -- and the step finishes the usual way.
// ---------------------------------------------------------------------------
struct StepCounters {
  long n_rk4, n_block_updates, n_refined, n_fam, memo_hits;
};

StepCounters counters_of(const mrb_ctx* c) {
  return StepCounters{c->n_rk4, c->n_block_updates, c->n_refined, c->n_fam, c->memo_hits};
}

void restore_counters(mrb_ctx* c, const StepCounters& k) {
  c->n_rk4 = k.n_rk4;
  c->n_block_updates = k.n_block_updates;
  c->n_refined = k.n_refined;
  c->n_fam = k.n_fam;
  c->memo_hits = k.memo_hits;
}

void switch_banks(mrb_ctx* c) {
  std::swap(c->h_part, c->h_part_b);
  std::swap(c->dpart, c->dpart_b);
  std::swap(c->part_st, c->part_st_b);
  std::swap(c->h_flags, c->h_flags_b);
  std::swap(c->dflags, c->dflags_b);
  std::swap(c->h_maxd, c->h_maxd_b);
  std::swap(c->dmaxd, c->dmaxd_b);
  std::swap(c->h_mq, c->h_mq_b);
  std::swap(c->dmq, c->dmq_b);
}

struct Issued {
  SpecSnap sn;
  std::vector<Leaf> pre;      // forest before the step
  std::vector<int> pre_free;
  char* pre_arena = nullptr;
  StepCounters cnt{};
  hipEvent_t ev = nullptr;
};

bool same_forest(const std::vector<Leaf>& a, const std::vector<Leaf>& b) {
  if (a.size() != b.size()) return false;
  for (size_t i = 0; i < a.size(); ++i)
    if (a[i].level != b[i].level || a[i].slot != b[i].slot || a[i].c[0] != b[i].c[0] || a[i].c[1] != b[i].c[1] ||
        a[i].c[2] != b[i].c[2])
      return false;
  return true;
}

// refinement, the one tile launch and the speculated coarsening of one step, without
// reading anything back: *state 1.  Where the step is not of that kind: *state 0 and
// nothing done, or *state 2 and the step done the usual way (the refinement had been
// applied when that showed).
mrb_status issue_step(mrb_ctx* c, double t, double dt, Issued& is, int* state) {
  *state = 0;
  if (!refine_foldable(c) || c->leaves.size() > kMemoMaxLeaves) return MRB_OK;
  // the refinement and the coarsening must both come from the memo (then the step is a
  // replay of host state): check before changing anything
  std::vector<int> mat;
  memo_material(c, 0, nullptr, mat);
  if (!memo_find(c, 0, mat)) return MRB_OK;
  is.pre = c->leaves;
  is.pre_free = c->free_slots;
  is.pre_arena = c->arena;
  is.cnt = counters_of(c);
  mrb_status r = do_refine_all(c, false);
  if (r) return r;
  if (!spec_all_merge(c)) {
    // the refinement is done but the step cannot be one launch: finish it the usual way
    if ((r = launch_refine_kernel(c, c->pending_ref, false))) return r;
    bool tiled = false;
    if ((r = rk4_adapt_tiled(c, t, dt, &tiled, false))) return r;
    if (!tiled && (r = do_rk4(c, t, dt))) return r;
    if (!tiled && (r = do_adapt(c, nullptr, false, false))) return r;
    *state = 2;
    return MRB_OK;
  }
  mrb_ctx::Memo* e = spec_entry(c);
  const int tn = c->ma_nsub > 0 ? c->ma_nsub : rk4t_pick(c), tpb = c->ma_nsub > 0 ? c->ma_tpb : 256;
  Rk4tArgs ra = rk4t_args(c, t, dt);
  c->flag_set = 0;
  rk4t_analysis_args(c, ra, e->smap);
  ra.mq = c->dmq;
  c->mq_parts = tn * tn;
  if ((r = launch_tiled(c, tn, ra, true, tpb, true, true))) return r;
  std::swap(c->u, c->unew);
  c->n_rk4++;
  c->n_block_updates += (long)nblk(c);
  if ((r = spec_begin(c, e, true, is.sn))) return r;
  HIPCHK(c, hipEventRecord(is.ev, c->stream));
  *state = 1;
  return MRB_OK;
}

// take back a queued step (its launch has finished or is waited for here)
mrb_status take_back(mrb_ctx* c, Issued& q) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::swap(c->u, c->unew);
  restore_counters(c, q.cnt);
  return MRB_OK;
}

// the second pass's flags would merge families (the memo's answer where it has one)
bool would_merge(mrb_ctx* c, const int8_t* flags) {
  if (c->leaves.size() <= kMemoMaxLeaves) {
    std::vector<int> mat;
    memo_material(c, 1, flags, mat);
    if (mrb_ctx::Memo* e = memo_find(c, 1, mat)) return e->nfam > 0;
  }
  return !coarsenable(c, flags).empty();
}

// up to nsteps steps with the next launch queued ahead; *done steps are complete on return
mrb_status steps_cycled(mrb_ctx* c, double t0, double dt, int nsteps, int* done) {
  *done = 0;
  if (nsteps < 2 || !c->ev_issue[0] || !c->h_flags_b || !c->h_mq_b) return MRB_OK;
  Issued is[2];
  is[0].ev = c->ev_issue[0];
  is[1].ev = c->ev_issue[1];
  int st = 0;
  mrb_status r = issue_step(c, t0, dt, is[0], &st);
  if (r) return r;
  if (st != 1) {
    if (st == 2) {
      c->n_steps++;
      *done = 1;
    }
    return MRB_OK;
  }
  for (int k = 0;; ++k) {
    Issued& cur = is[k & 1];
    Issued& nxt = is[(k + 1) & 1];
    // queue the next step if this one returned the forest to where it started (then the
    // next step replays the same memoised transitions)
    bool queued = false;
    if (k + 1 < nsteps && c->arena == cur.pre_arena && same_forest(c->leaves, cur.pre) &&
        c->free_slots == cur.pre_free) {
      switch_banks(c);
      if ((r = issue_step(c, t0 + (k + 1) * dt, dt, nxt, &st))) return r;
      if (st != 1) return fail(c, MRB_E_STATE, "a cycling step could not be queued");
      queued = true;
      ++c->n_queued;
    }
    if (queued) switch_banks(c);   // this step's outputs
    {
      HostTimer ht(&c->hus_wait);
      HIPCHK(c, hipEventSynchronize(cur.ev));
    }
    ana_combine(c);
    bool keep = true;
    if (queued) {
      const bool hit = std::equal(c->h_flags, c->h_flags + cur.sn.n1, c->spec_flags.begin());
      if (hit) mother_flags(c);
      keep = hit && !would_merge(c, c->h_flags2);
      if (!keep) {
        if ((r = take_back(c, nxt))) return r;
        ++c->n_taken_back;
      }
    }
    if ((r = spec_finish(c, cur.sn, true, nullptr))) return r;
    c->n_steps++;
    ++*done;
    if (!queued || !keep) return MRB_OK;
    switch_banks(c);   // the queued step's outputs again
  }
}

mrb_status ensure_scratch(mrb_ctx* c, size_t bytes) {
  if (bytes <= c->scratch_cap) return MRB_OK;
  if (c->dscratch) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipFree(c->dscratch));
    c->dscratch = nullptr;
  }
  HIPCHK(c, hipMalloc(&c->dscratch, bytes));
  c->scratch_cap = bytes;
  return MRB_OK;
}

bool check_state(mrb_ctx* c, bool need_data) {
  if (!c->have_forest) { c->err = "no forest (call mrb_init_forest first)"; return false; }
  if (need_data && !c->have_data) { c->err = "no block data (call mrb_load_blocks first)"; return false; }
  return true;
}

}  // namespace

// scatter/gather of whole blocks between a contiguous array and pool slots
namespace mrb {
hipError_t launch_scatter(const double* src, const int* slots, int n, size_t bsz, double* dst, hipStream_t st);
}

namespace {

// One MR step with the refinement, the four stages and the first analysis replayed
// from a captured graph (launch parameters are fixed; block counts and
// descriptors come from the device topology header).
mrb_status step_graph(mrb_ctx* c, double t, double dt) {
  mrb_status r = do_refine_all(c, false);
  if (r) return r;
  uint64_t dtb;
  std::memcpy(&dtb, &dt, sizeof dtb);
  const int ns = pick_nsub(c);
  const int nsm = pick_aux(c, (long)c->hblk.size(), c->nsub_mr);
  const int nsr = pick_aux(c, (long)std::max(1, c->pending_ref) << c->cfg.dim, c->nsub_ref);
  // the first analysis pass writes the speculated coarsening's mothers when there is one
  // (its map is read at replay time from the memo's device copy)
  mrb_ctx::Memo* se = spec_entry(c);
  const int* smap = se ? se->smap : nullptr;
  // the launches take the topology header by value: a replay needs the same header
  uint64_t key[7 + sizeof(TopoHeader) / 8] = {
      (uint64_t)(uintptr_t)c->u, (uint64_t)ns | ((uint64_t)c->order << 8) | ((uint64_t)pick_tpb(c, ns) << 16),
      (uint64_t)nsm, (uint64_t)nsr, dtb, (uint64_t)(uintptr_t)c->arena, (uint64_t)(uintptr_t)smap};
  std::memcpy(key + 7, &c->arena_hdr, sizeof(TopoHeader));
  hipGraphExec_t exec = nullptr;
  for (auto& g : c->graphs)
    if (std::memcmp(g.key, key, sizeof key) == 0) exec = g.exec;
  if (!exec) {
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    mrb_status e = launch_refine_kernel(c, std::max(1, c->pending_ref), true);
    if (!e) e = sweep(c, t, dt, true);
    double* u0 = c->u;
    if (!e) {
      std::swap(c->u, c->unew);
      e = launch_mr_kernel(c, true, smap ? se : nullptr);
      std::swap(c->u, c->unew);
    }
    hipGraph_t graph = nullptr;
    hipError_t ec = hipStreamEndCapture(c->stream, &graph);
    if (e) { if (graph) (void)hipGraphDestroy(graph); return e; }
    if (ec != hipSuccess) return fail(c, MRB_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ec != hipSuccess) return fail(c, MRB_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ec));
    (void)u0;
    if (c->graphs.size() >= 4) {
      (void)hipGraphExecDestroy(c->graphs.front().exec);
      c->graphs.erase(c->graphs.begin());
    }
    mrb_ctx::GraphEntry ge;
    std::memcpy(ge.key, key, sizeof key);
    ge.exec = exec;
    c->graphs.push_back(ge);
  }
  {
    HostTimer ht(&c->hus_launch);
    HIPCHK(c, hipGraphLaunch(exec, c->stream));
  }
  c->n_graph_launches++;
  std::swap(c->u, c->unew);
  c->n_rk4++;
  c->n_block_updates += (long)c->hblk.size();
  return do_adapt(c, nullptr, true, smap != nullptr);
}

// The synchronised solution on the uniform lattice of `level` into device memory dst
// ([nf][N^dim], x fastest).  Every lattice point is a node of the finest leaf holding
// it once no leaf is coarser than `level`, so leaves below `level` are refined first --
// level by level, into free pool slots, with the refinement kernel, whose children take
// the synchronised finer values (prediction where no leaf holds a node) -- on a copy of
// the forest: the refinement writes only new slots, the solver's own slots are never
// handed out, and the host forest and the device topology are put back afterwards.
mrb_status read_uniform_to(mrb_ctx* c, int level, double* dst) {
  const int nch = 1 << c->cfg.dim;
  bool deeper = false;
  for (const Leaf& L : c->leaves) deeper = deeper || L.level < level;
  if (!deeper) {
    ReadArgs a{topo(c), c->u, dst, level};
    HIPCHK(c, launch_read(c->shape, grid_for(c, (long)c->leaves.size()), a, c->stream));
    return MRB_OK;
  }
  // state to put back
  std::vector<Leaf> leaves0 = c->leaves;
  std::vector<BlockDesc> hblk0 = c->hblk;
  std::vector<NbEntry> hnb0 = c->hnb;
  std::vector<int> hlist0 = c->hlist, level0 = c->level_off, free0 = c->free_slots;
  const long n_refined0 = c->n_refined;
  const bool have_flags0 = c->have_flags;
  std::vector<char> own((size_t)c->cfg.max_blocks, 0);
  for (const Leaf& L : c->leaves) own[(size_t)L.slot] = 1;
  mrb_status s = MRB_OK;
  for (;;) {
    std::vector<int> par;
    for (int i = 0; i < (int)c->leaves.size(); ++i)
      if (c->leaves[i].level < level) par.push_back(i);
    if (par.empty()) break;
    if (c->free_slots.size() < par.size() * (size_t)nch) {
      s = fail(c, MRB_E_CAPACITY, "read_uniform: the pool has too few free slots to refine to this level");
      break;
    }
    if ((s = do_refine(c, par, true, false))) break;
    // slots of the solver's own blocks return to the free list as parents: keep them out
    c->free_slots.erase(std::remove_if(c->free_slots.begin(), c->free_slots.end(),
                                       [&](int sl) { return own[(size_t)sl] != 0; }),
                        c->free_slots.end());
  }
  if (!s) {
    ReadArgs a{topo(c), c->u, dst, level};
    if (hipError_t e = launch_read(c->shape, grid_for(c, (long)c->leaves.size()), a, c->stream))
      s = fail(c, MRB_E_DEVICE, std::string("read_uniform: ") + hipGetErrorString(e));
  }
  // the kernels above read the topology buffer that the restore below overwrites
  hipError_t es = hipStreamSynchronize(c->stream);
  c->leaves.swap(leaves0);
  c->index.clear();
  for (size_t i = 0; i < c->leaves.size(); ++i) c->index.set(pack_key(c->leaves[i].level, c->leaves[i].c), (int)i);
  c->hblk.swap(hblk0);
  c->hnb.swap(hnb0);
  c->hlist.swap(hlist0);
  c->level_off.swap(level0);
  c->free_slots.swap(free0);
  c->n_refined = n_refined0;
  c->pending_ref = 0;
  c->hcount_ref_zero = true;
  mrb_status su = upload_topo(c);
  c->have_flags = have_flags0;
  if (s) return s;
  if (es != hipSuccess) return fail(c, MRB_E_DEVICE, std::string("read_uniform: ") + hipGetErrorString(es));
  return su;
}

// ---------------------------------------------------------------------------
// device-resident topology (the plan kernels are in topo.hip)
// ---------------------------------------------------------------------------

// Arena layout of the device path: fixed offsets for max_blocks blocks and entry rows of
// the largest possible entry count, so a plan kernel can write a grid whose size the
// host learns only afterwards.
TopoHeader dev_header(const mrb_ctx* c, int n, int nref, int nfam) {
  TopoHeader h;
  std::memset(&h, 0, sizeof h);
  const size_t cap = (size_t)c->cfg.max_blocks, S = (size_t)c->dev.stride;
  size_t off = align16(sizeof(TopoHeader));
  auto place = [&](size_t bytes) {
    const size_t o = off;
    off = align16(off + bytes);
    return (int)o;
  };
  h.off_blk = place(cap * sizeof(BlockDesc));
  h.off_nb = place(cap * S * sizeof(NbEntry));
  h.off_list = place(cap * sizeof(int));
  h.off_pblk = place(cap * sizeof(BlockDesc));
  h.off_pnb = place(cap * S * sizeof(NbEntry));
  h.off_ref = place(cap * sizeof(RefineDesc));
  h.off_fam = place(cap * sizeof(FamilyDesc));
  h.nb_stride = h.pnb_stride = (int)S;
  h.n_blocks = n;
  h.n_ref = h.n_pblk = nref;
  h.n_fam = nfam;
  h.pad[0] = (int)std::min(off, (size_t)0x7fffffff);   // bytes of the layout (host bookkeeping only)
  return h;
}

// allocate the device path's buffers once; false (with dev.unavailable) if the dense
// index of every possible block would not fit
mrb_status dev_alloc(mrb_ctx* c) {
  auto& D = c->dev;
  if (D.ready) return MRB_OK;
  const int d = c->cfg.dim;
  size_t cells = 0;
  for (int l = 0; l <= c->cfg.jmax + 1 && l <= kMaxLevels; ++l) {
    D.cell_off[l] = (int)cells;
    if (l >= 1 && l <= c->cfg.jmax) cells += (size_t)1 << (d * l);
    if (cells > ((size_t)1 << 26)) {
      D.unavailable = true;
      return fail(c, MRB_E_ARG, "device topology: the dense block index of this jmax does not fit");
    }
  }
  D.ncells = cells;
  D.stride = d == 2 ? 13 : 57;
  const TopoHeader h = dev_header(c, 0, 0, 0);
  const size_t ab = (size_t)h.pad[0];
  if (ab >= (size_t)0x7fffffff) return fail(c, MRB_E_CAPACITY, "device topology: arena exceeds 2 GiB");
  const size_t mb = (size_t)c->cfg.max_blocks;
  HIPCHK(c, hipMalloc((void**)&D.arena[0], ab));
  HIPCHK(c, hipMalloc((void**)&D.arena[1], ab));
  HIPCHK(c, hipMalloc((void**)&D.cells, cells * sizeof(int)));
  HIPCHK(c, hipMalloc((void**)&D.stack, mb * sizeof(int)));
  HIPCHK(c, hipMalloc((void**)&D.scratch, 3 * mb * sizeof(int)));
  HIPCHK(c, hipMalloc((void**)&D.edges, (2 + 2 * mb * (size_t)D.stride) * sizeof(int)));
  HIPCHK(c, hipMalloc((void**)&D.err, 256));
  HIPCHK(c, hipMemset(D.err, 0, 256));
  HIPCHK(c, hipMalloc((void**)&D.flags, std::max(mb, (size_t)256)));
  HIPCHK(c, hipMalloc((void**)&D.maxd, std::max(mb * c->cfg.nfields * sizeof(double), (size_t)256)));
  HIPCHK(c, hipHostMalloc((void**)&D.h_out, kDevOutInts * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
  HIPCHK(c, hipHostGetDevicePointer((void**)&D.d_out, D.h_out, 0));
  D.arena_bytes = ab;
  D.ready = true;
  return MRB_OK;
}

void dev_release(mrb_ctx* c) {
  auto& D = c->dev;
  release_staging(D.st_blk);
  release_staging(D.st_stack);
  void* p[] = {D.arena[0], D.arena[1], D.cells, D.stack, D.scratch, D.edges, D.err, D.flags, D.maxd};
  for (void* q : p)
    if (q) (void)hipFree(q);
  if (D.h_out) (void)hipHostFree(D.h_out);
}

DevTopoArgs dev_args(mrb_ctx* c, int from, const TopoHeader& oh, int to, const TopoHeader& nh) {
  auto& D = c->dev;
  DevTopoArgs a;
  std::memset(&a, 0, sizeof a);
  a.old_base = D.arena[from];
  a.old_h = oh;
  a.new_base = D.arena[to];
  a.new_h = nh;
  a.cells = D.cells;
  for (int l = 0; l <= kMaxLevels; ++l) a.cell_off[l] = D.cell_off[std::min(l, c->cfg.jmax + 1)];
  a.free_stack = D.stack;
  a.free_top = D.top;
  a.flags = D.flags;
  a.maxd = D.maxd;
  a.nf = c->cfg.nfields;
  a.scratch = D.scratch;
  a.edges = D.edges;
  a.err = D.err;
  a.out = D.d_out;
  a.dim = c->cfg.dim;
  a.bs = c->cfg.bs;
  a.jmax = c->cfg.jmax;
  a.nch = 1 << c->cfg.dim;
  return a;
}

int dev_grid(long waves) { return (int)std::max(1L, std::min(8192L, (waves + 3) / 4)); }

// the device takes over the host forest: descriptors and free stack uploaded, dense
// index and entries built on the device
mrb_status dev_push(mrb_ctx* c) {
  auto& D = c->dev;
  if (mrb_status s = dev_alloc(c)) return s;
  HostTimer ht(&c->hus_upload);
  const int n = (int)c->leaves.size();
  std::vector<BlockDesc> bd(n);
  for (int i = 0; i < n; ++i) {
    const Leaf& L = c->leaves[i];
    bd[i].slot = L.slot;
    bd[i].level = L.level;
    for (int a = 0; a < 3; ++a) bd[i].c[a] = L.c[a];
    bd[i].nb_begin = bd[i].n_ent = bd[i].n_coarse = 0;
  }
  D.cur = 0;
  const TopoHeader h = dev_header(c, n, 0, 0);
  if (mrb_status s = stage_upload(c, D.st_blk, bd.data(), n * sizeof(BlockDesc), D.arena[D.cur] + h.off_blk)) return s;
  if (!c->free_slots.empty())
    if (mrb_status s = stage_upload(c, D.st_stack, c->free_slots.data(), c->free_slots.size() * sizeof(int), D.stack))
      return s;
  HIPCHK(c, launch_fill_int(D.cells, D.ncells, -1, c->stream));
  D.top = (int)c->free_slots.size();
  D.n = n;
  for (int l = 0; l < kMaxLevels; ++l) D.hist[l] = 0;
  for (const Leaf& L : c->leaves) D.hist[L.level]++;
  DevTopoArgs a = dev_args(c, D.cur, h, D.cur, h);
  {
    TimeScope ts(c, T_TOPO, 0.0);
    HIPCHK(c, launch_index(a, 1, dev_grid(4L * n), c->stream));
    HIPCHK(c, launch_entries(a, dev_grid(n), c->stream));
  }
  c->arena = D.arena[D.cur];
  c->arena_hdr = h;
  c->pending_ref = 0;
  D.have_flags = false;
  D.active = true;
  D.pushes++;
  return MRB_OK;
}

// the host takes the forest back from the device: descriptors and free stack
// downloaded, host entries rebuilt and uploaded, flags of the last analysis kept
mrb_status dev_pull(mrb_ctx* c) {
  auto& D = c->dev;
  if (!D.active) return MRB_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int err = 0;
  HIPCHK(c, hipMemcpy(&err, D.err, sizeof(int), hipMemcpyDeviceToHost));
  if (err & 1) return fail(c, MRB_E_TOPOLOGY, "device topology: a grid was not graded");
  const TopoHeader h = c->arena_hdr;
  std::vector<BlockDesc> bd(D.n);
  std::vector<int> stack(D.top);
  HIPCHK(c, hipMemcpy(bd.data(), D.arena[D.cur] + h.off_blk, D.n * sizeof(BlockDesc), hipMemcpyDeviceToHost));
  if (D.top) HIPCHK(c, hipMemcpy(stack.data(), D.stack, D.top * sizeof(int), hipMemcpyDeviceToHost));
  std::vector<int8_t> fl;
  std::vector<double> md;
  if (D.have_flags) {
    fl.resize(D.n);
    md.resize((size_t)D.n * c->cfg.nfields);
    HIPCHK(c, hipMemcpy(fl.data(), D.flags, D.n, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(md.data(), D.maxd, md.size() * sizeof(double), hipMemcpyDeviceToHost));
  }
  c->leaves.resize(D.n);
  for (int i = 0; i < D.n; ++i) {
    Leaf& L = c->leaves[i];
    L.level = bd[i].level;
    for (int a = 0; a < 3; ++a) L.c[a] = bd[i].c[a];
    L.slot = bd[i].slot;
  }
  c->free_slots.swap(stack);
  D.active = false;
  D.pulls++;
  sort_and_index(c);   // the device order is the forest order already; keys and index rebuilt
  if (mrb_status s = build_descriptors(c)) return s;
  c->hcount_ref_zero = true;
  c->pending_ref = 0;
  if (mrb_status s = upload_topo(c)) return s;
  if (D.have_flags) {
    c->last_flags.assign(fl.begin(), fl.end());
    c->last_maxd.assign(md.begin(), md.end());
    c->have_flags = true;
  }
  return MRB_OK;
}

// the safety-zone refinement planned and run on the device
mrb_status dev_refine_all(mrb_ctx* c) {
  auto& D = c->dev;
  const int nch = 1 << c->cfg.dim;
  const int nref = D.n - (int)D.hist[c->cfg.jmax];
  c->pending_ref = 0;
  if (nref == 0) return MRB_OK;
  if (D.top < nref * nch) return fail(c, MRB_E_CAPACITY, "refine_all: pool too small");
  const int nnew = D.n + nref * (nch - 1), nxt = D.cur ^ 1;
  const TopoHeader nh = dev_header(c, nnew, nref, 0);
  DevTopoArgs a = dev_args(c, D.cur, c->arena_hdr, nxt, nh);
  {
    TimeScope ts(c, T_TOPO, 0.0);
    HIPCHK(c, launch_plan_refine(a, c->stream));
    HIPCHK(c, launch_index(a, 0, dev_grid(4L * D.n), c->stream));
    HIPCHK(c, launch_index(a, 1, dev_grid(4L * nnew), c->stream));
    HIPCHK(c, launch_entries(a, dev_grid((long)nnew + nref), c->stream));
  }
  long h2[kMaxLevels] = {0};
  for (int l = 1; l < kMaxLevels; ++l) {
    if (l < c->cfg.jmax) h2[l + 1] += D.hist[l] * nch;
    else h2[l] += D.hist[l];
  }
  for (int l = 0; l < kMaxLevels; ++l) D.hist[l] = h2[l];
  D.top = D.top - nref * nch + nref;
  D.n = nnew;
  D.cur = nxt;
  D.have_flags = false;
  c->arena = D.arena[D.cur];
  c->arena_hdr = nh;
  c->pending_ref = nref;
  c->n_refined += nref;
  c->have_flags = false;
  return launch_refine_kernel(c, nref, false);
}

// analysis and coarsening until nothing merges, planned on the device; one read-back
// of a few counts per pass
mrb_status dev_adapt(mrb_ctx* c, int* npass) {
  auto& D = c->dev;
  const int nch = 1 << c->cfg.dim;
  int passes = 0;
  for (;;) {
    {
      const int n = D.n;
      MrArgs m = mr_args(c);
      m.flags = D.flags;
      m.maxd = D.maxd;
      const int ns = pick_aux(c, n, c->nsub_mr);
      long work = n;
      for (int q = 0; q < c->cfg.dim; ++q) work *= ns;
      TimeScope ts(c, T_MR, (double)n * c->bsz * 8.0);
      HIPCHK(c, launch_mr(c->shape, ns, mr_tpb(c, ns), grid_for(c, work), m, c->stream));
    }
    ++passes;
    c->n_mr++;
    D.passes++;
    const int nxt = D.cur ^ 1;
    DevTopoArgs a = dev_args(c, D.cur, c->arena_hdr, nxt, dev_header(c, 0, 0, 0));
    {
      TimeScope ts(c, T_TOPO, 0.0);
      HIPCHK(c, launch_plan_coarsen(a, dev_grid((long)D.n * D.stride / 16), c->stream));
    }
    {
      HostTimer ht(&c->hus_wait);
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if (mrb_status r = check_barrier(c)) return r;
    const int m = D.h_out[0], nnew = D.h_out[1], top = D.h_out[2], err = D.h_out[3];
    D.have_flags = true;
    c->have_flags = false;
    if (err & 1) return fail(c, MRB_E_TOPOLOGY, "device topology: a grid was not graded");
    if (err & 2) return fail(c, MRB_E_NONFINITE, "detail norm is not finite");
    if (err & 4) return fail(c, MRB_E_CAPACITY, "coarsen: pool too small");
    if (m == 0) break;
    if (passes > c->cfg.jmax + 2) return fail(c, MRB_E_STATE, "adapt did not reach a fixed point");
    if (nnew != D.n - m * (nch - 1)) return fail(c, MRB_E_STATE, "device topology: inconsistent coarsening counts");
    const TopoHeader nh = dev_header(c, nnew, 0, m);
    a = dev_args(c, D.cur, c->arena_hdr, nxt, nh);
    {
      TimeScope ts(c, T_TOPO, 0.0);
      HIPCHK(c, launch_index(a, 0, dev_grid(4L * D.n), c->stream));
      HIPCHK(c, launch_index(a, 1, dev_grid(4L * nnew), c->stream));
      HIPCHK(c, launch_entries(a, dev_grid(nnew), c->stream));
    }
    for (int l = 0; l < kMaxLevels; ++l) D.hist[l] = D.h_out[4 + l];
    D.top = top;
    D.n = nnew;
    D.cur = nxt;
    D.have_flags = false;
    c->arena = D.arena[D.cur];
    c->arena_hdr = nh;
    c->n_fam += m;
    CoarsenArgs ca{topo(c), c->u};
    const long total = (long)m * c->np;
    TimeScope ts(c, T_COARSEN, (double)total * c->cfg.nfields * 16.0);
    HIPCHK(c, launch_coarsen(c->shape, (int)std::min(4096L, (total + 255) / 256), ca, c->stream));
  }
  if (npass) *npass = passes;
  return MRB_OK;
}

// whether mrb_step plans on the device: fused form, a dense index that fits, and mode 1,
// or mode 2 with a refined grid above the memo limit
bool want_device(mrb_ctx* c) {
  auto& D = c->dev;
  if (D.mode == 0 || D.unavailable || c->cfg.form != MRB_FORM_FUSED) return false;
  if (D.mode == 1) return true;
  const long n = (long)nblk(c);
  long below = 0;
  if (D.active) below = n - D.hist[c->cfg.jmax];
  else
    for (const Leaf& L : c->leaves) below += L.level < c->cfg.jmax;
  return n + below * ((1L << c->cfg.dim) - 1) > (long)kMemoMaxLeaves;
}

bool graph_ok(const mrb_ctx* c) {
  return c->use_graph && !c->timing && c->cfg.form == MRB_FORM_FUSED && !filter_on(c) &&
         !(c->cfg.physics == MRB_ADV_SWIRL && c->cfg.phys[0] > 0.0) && c->stream != nullptr;
}

}  // namespace

extern "C" {

const char* mrb_last_error(const mrb_ctx* c) { return c ? c->err.c_str() : "null context"; }

mrb_status mrb_create(const mrb_config* cfg, double* u, double* u_new, void* k1, void* k2, void* k3, void* stream,
                      mrb_ctx** out) {
  if (!out || !cfg) return MRB_E_ARG;
  *out = nullptr;
  mrb_ctx* c = new mrb_ctx();
  c->cfg = *cfg;
  c->cfg.swirl_s2 = c->cfg.swirl_s = c->cfg.field_scale = c->cfg.field_offset = nullptr;
  auto bad = [&](const char* m) {
    c->err = m;
    *out = c;  // hand back the context so the caller can read the message
    return MRB_E_ARG;
  };
  if (!u || !u_new || !k1 || !k2 || !k3) return bad("pool pointers must be non-null");
  if (cfg->dim < 2 || cfg->dim > 3) return bad("dim must be 2 or 3");
  if (cfg->bs < 5 || cfg->bs % 2 == 0 || cfg->bs > 63) return bad("bs must be odd, 5..63");
  if (cfg->hw < 2 || cfg->hw % 2) return bad("hw must be even and >= 2");
  if ((cfg->bs - 1) / 2 < cfg->hw + 2) return bad("need (bs-1)/2 >= hw + 2");
  if (cfg->nfields < 1 || cfg->nfields > 4) return bad("nfields must be 1..4");
  if (cfg->jmax < 2 || cfg->jmax >= kMaxLevels - 1) return bad("jmax out of range");
  if (cfg->max_blocks < (1 << cfg->dim)) return bad("max_blocks too small");
  {
    size_t npt = 1;
    for (int a = 0; a < cfg->dim; ++a) npt *= (size_t)cfg->bs;
    // the kernels address the pool with 32-bit offsets
    if ((size_t)cfg->max_blocks * (size_t)cfg->nfields * npt >= ((size_t)1 << 31))
      return bad("max_blocks * nfields * bs^dim must stay below 2^31");
  }
  if (cfg->precision != MRB_FP64 && cfg->precision != MRB_MIXED) return bad("precision");
  if (cfg->form != MRB_FORM_PLAIN && cfg->form != MRB_FORM_FUSED) return bad("form");
  if (cfg->form == MRB_FORM_PLAIN && cfg->precision != MRB_FP64) return bad("the plain form is FP64 only");
  if (cfg->physics < 0 || cfg->physics > 2) return bad("physics");
  if (cfg->physics == MRB_ADV_SWIRL && (cfg->dim != 2 || !cfg->swirl_s2 || !cfg->swirl_s))
    return bad("swirl needs dim 2 and both tables");
  if ((cfg->physics == MRB_NS2D) != (cfg->nfields == 4) || (cfg->physics == MRB_NS2D && (cfg->dim != 2 || cfg->hw != 4)))
    return bad("Navier-Stokes needs dim 2, hw 4 and 4 fields (and only it has 4 fields)");
  if (cfg->physics == MRB_NS2D && (cfg->phys[0] <= 1.0 || cfg->phys[1] < 0.0 || cfg->phys[2] <= 0.0 ||
                                    !(cfg->phys[3] >= 0.0)))
    return bad("Navier-Stokes needs gamma > 1, mu >= 0, Pr > 0 and a filter threshold >= 0");
  c->shape = Shape{cfg->dim, cfg->bs, cfg->hw, cfg->nfields};
  if (!shape_supported(c->shape)) return bad("unsupported (dim, bs, hw, nfields) combination");
  c->np = 1;
  for (int a = 0; a < cfg->dim; ++a) c->np *= cfg->bs;
  c->bsz = (size_t)cfg->nfields * c->np;
  c->stream = (hipStream_t)stream;
  c->u = u;
  c->unew = u_new;
  c->k[0] = k1;
  c->k[1] = k2;
  c->k[2] = k3;
  for (int f = 0; f < cfg->nfields; ++f) {
    c->thr.push_back(cfg->field_scale ? cfg->eps * cfg->field_scale[f] : cfg->eps);
    c->off.push_back(cfg->field_offset && cfg->precision == MRB_MIXED ? cfg->field_offset[f] : 0.0);
  }
  for (int l = 0; l < kMaxLevels; ++l) {
    const long nl = l >= 1 ? (1L << l) * (cfg->bs - 1) : (cfg->bs - 1);
    c->lt.nl[l] = (int)nl;
    c->lt.r[l] = (double)nl / 12.0;
    c->lt.rf[l] = (float)c->lt.r[l];
  }
  std::memset(&c->ph, 0, sizeof c->ph);
  c->ph.kind = cfg->physics;
  c->ph.jmax = cfg->jmax;
  for (int a = 0; a < 3; ++a) c->ph.c[a] = cfg->phys[a];
  if (cfg->physics == MRB_NS2D) {
    const double gam = cfg->phys[0], mu = cfg->phys[1], pr = cfg->phys[2];
    c->ph.gamma = gam;
    c->ph.mu = mu;
    c->ph.kap = mu * gam / ((gam - 1.0) * pr);
  }
  c->index.init(cfg->dim, cfg->jmax);
  auto dev = [&](void** p, size_t bytes) -> bool {
    hipError_t e = hipMalloc(p, std::max(bytes, (size_t)256));
    if (e != hipSuccess) { c->err = std::string("hipMalloc: ") + hipGetErrorString(e); return false; }
    return true;
  };
  const size_t mb = cfg->max_blocks;
  bool ok = dev((void**)&c->dacc, mb * cfg->nfields * 8) && dev((void**)&c->ddone, mb * sizeof(int)) &&
            hipMemset(c->dacc, 0, mb * cfg->nfields * 8) == hipSuccess &&
            hipMemset(c->ddone, 0, mb * sizeof(int)) == hipSuccess && dev((void**)&c->dslots, mb * sizeof(int));
  if (ok && cfg->physics == MRB_ADV_SWIRL) {
    const size_t n = (size_t)(1L << cfg->jmax) * (cfg->bs - 1);
    ok = dev((void**)&c->ds2, n * sizeof(double)) && dev((void**)&c->ds, n * sizeof(double));
    if (ok) {
      ok = hipMemcpy(c->ds2, cfg->swirl_s2, n * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(c->ds, cfg->swirl_s, n * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
      if (!ok) c->err = "copying swirl tables failed";
    }
    c->ph.s2 = c->ds2;
    c->ph.s = c->ds;
  }
  if (ok && cfg->form == MRB_FORM_PLAIN) {
    size_t g = 1;
    for (int a = 0; a < cfg->dim; ++a) g *= (size_t)(cfg->bs + 2 * cfg->hw);
    ok = dev((void**)&c->dghost, mb * cfg->nfields * g * sizeof(double));
  }
  if (ok) {
    // flags and detail maxima go straight from the analysis kernel into mapped,
    // coherent host memory: reading them back is one stream synchronisation
    const unsigned fl = hipHostMallocMapped | hipHostMallocCoherent;
    ok = hipHostMalloc((void**)&c->h_flags, mb, fl) == hipSuccess &&
         hipHostMalloc((void**)&c->h_maxd, mb * cfg->nfields * sizeof(double), fl) == hipSuccess &&
         hipHostGetDevicePointer((void**)&c->dflags, c->h_flags, 0) == hipSuccess &&
         hipHostGetDevicePointer((void**)&c->dmaxd, c->h_maxd, 0) == hipSuccess &&
         hipHostMalloc((void**)&c->h_flags2, mb, fl) == hipSuccess &&
         hipHostMalloc((void**)&c->h_maxd2, mb * cfg->nfields * sizeof(double), fl) == hipSuccess &&
         hipHostGetDevicePointer((void**)&c->dflags2, c->h_flags2, 0) == hipSuccess &&
         hipHostGetDevicePointer((void**)&c->dmaxd2, c->h_maxd2, 0) == hipSuccess &&
         hipHostMalloc((void**)&c->h_err, sizeof(int), fl) == hipSuccess &&
         hipHostGetDevicePointer((void**)&c->d_err, c->h_err, 0) == hipSuccess &&
         (cfg->dim != 2 || cfg->nfields != 1 ||
          (hipHostMalloc((void**)&c->h_mq, mb * 16 * sizeof(double), fl) == hipSuccess &&
           hipHostGetDevicePointer((void**)&c->dmq, c->h_mq, 0) == hipSuccess &&
           hipHostMalloc((void**)&c->h_mq_b, mb * 16 * sizeof(double), fl) == hipSuccess &&
           hipHostGetDevicePointer((void**)&c->dmq_b, c->h_mq_b, 0) == hipSuccess &&
           hipHostMalloc((void**)&c->h_flags_b, mb, fl) == hipSuccess &&
           hipHostGetDevicePointer((void**)&c->dflags_b, c->h_flags_b, 0) == hipSuccess &&
           hipHostMalloc((void**)&c->h_maxd_b, mb * sizeof(double), fl) == hipSuccess &&
           hipHostGetDevicePointer((void**)&c->dmaxd_b, c->h_maxd_b, 0) == hipSuccess &&
           hipHostMalloc((void**)&c->h_part, mb * 16 * sizeof(double), fl) == hipSuccess &&
           hipHostGetDevicePointer((void**)&c->dpart, c->h_part, 0) == hipSuccess &&
           hipHostMalloc((void**)&c->h_part_b, mb * 16 * sizeof(double), fl) == hipSuccess &&
           hipHostGetDevicePointer((void**)&c->dpart_b, c->h_part_b, 0) == hipSuccess &&
           hipEventCreateWithFlags(&c->ev_issue[0], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&c->ev_issue[1], hipEventDisableTiming) == hipSuccess));
    if (!ok) c->err = "hipHostMalloc (mapped) failed";
    if (ok) *c->h_err = 0;
    ok = ok && dev((void**)&c->dbar, kBarWords * sizeof(unsigned)) &&
         hipMemset(c->dbar, 0, kBarWords * sizeof(unsigned)) == hipSuccess;
  }
  if (ok) {
    // looked up once per device here; a failure only disables mrb_mr_pass_noalloc
    hipError_t e = scratch_setup(&c->scratch_dev);
    if (e != hipSuccess) c->scratch_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    c->last_flags.reserve(mb);
    c->last_maxd.reserve(mb * cfg->nfields);
  }
  if (ok) {
    int dev_id = 0, ncu = 0;
    (void)hipGetDevice(&dev_id);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev_id) == hipSuccess && ncu > 0) {
      c->ncu = ncu;
      c->grid = ncu * 8;
    }
  }
  *out = c;
  if (!ok) return MRB_E_DEVICE;
  return MRB_OK;
}

mrb_status mrb_destroy(mrb_ctx* c) {
  if (!c) return MRB_E_ARG;
  (void)hipStreamSynchronize(c->stream);
  Staging* sts[] = {&c->st_topo[0], &c->st_topo[1], &c->st_slots};
  for (Staging* s : sts) release_staging(*s);
  for (auto& t : c->timed) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  void* mlpbufs[] = {c->mp, c->mgrad, c->mm, c->mv, c->mnorm, c->mx, c->mxn, c->mz1, c->ma1, c->mz2, c->ma2,
                     c->mlog, c->mloss, c->mdl, c->mdz1, c->mdz2, c->mcw, c->mpmax, c->my, c->mpred};
  for (void* p : mlpbufs)
    if (p) (void)hipFree(p);
  for (auto& e : c->memo)
    if (e.arena) (void)hipFree(e.arena);
  dev_release(c);
  void* ptrs[] = {c->work_arena, c->dacc, c->ddone,
                  c->ds2, c->ds, c->dghost, c->dscratch, c->dslots, c->dbar};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->h_flags) (void)hipHostFree(c->h_flags);
  if (c->h_maxd) (void)hipHostFree(c->h_maxd);
  if (c->h_flags2) (void)hipHostFree(c->h_flags2);
  if (c->h_maxd2) (void)hipHostFree(c->h_maxd2);
  if (c->h_err) (void)hipHostFree(c->h_err);
  if (c->h_mq) (void)hipHostFree(c->h_mq);
  if (c->h_mq_b) (void)hipHostFree(c->h_mq_b);
  if (c->h_part) (void)hipHostFree(c->h_part);
  if (c->h_part_b) (void)hipHostFree(c->h_part_b);
  if (c->h_flags_b) (void)hipHostFree(c->h_flags_b);
  if (c->h_maxd_b) (void)hipHostFree(c->h_maxd_b);
  for (hipEvent_t ev : c->ev_issue)
    if (ev) (void)hipEventDestroy(ev);
  delete c;
  return MRB_OK;
}

mrb_status mrb_init_forest(mrb_ctx* c, int n, const int8_t* level, const int32_t* coords) {
  if (!c) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (n <= 0 || !level || !coords) return fail(c, MRB_E_ARG, "init_forest: empty forest or null arrays");
  if (n > c->cfg.max_blocks) return fail(c, MRB_E_CAPACITY, "init_forest: more blocks than max_blocks");
  const int d = c->cfg.dim;
  // a rejected forest leaves the previous state unchanged
  std::vector<Leaf> old_leaves;
  old_leaves.swap(c->leaves);
  auto old_index = c->index;
  auto restore = [&](mrb_status s) {
    c->leaves.swap(old_leaves);
    c->index = old_index;
    return s;
  };
  for (int i = 0; i < n; ++i) {
    Leaf L;
    L.level = level[i];
    L.c[0] = L.c[1] = L.c[2] = 0;
    if (L.level < 1 || L.level > c->cfg.jmax) return restore(fail(c, MRB_E_TOPOLOGY, "level out of range"));
    for (int a = 0; a < d; ++a) {
      L.c[a] = coords[(size_t)i * d + a];
      if (L.c[a] < 0 || L.c[a] >= (1 << L.level)) return restore(fail(c, MRB_E_TOPOLOGY, "coords out of range"));
    }
    L.slot = -1;
    c->leaves.push_back(L);
  }
  sort_and_index(c);
  if (c->index.size() != c->leaves.size()) return restore(fail(c, MRB_E_TOPOLOGY, "duplicate block"));
  mrb_status s = check_forest(c);
  if (s) return restore(s);
  for (int i = 0; i < n; ++i) c->leaves[i].slot = i;
  if ((s = build_descriptors(c))) return restore(s);
  c->free_slots.clear();
  for (int sl = c->cfg.max_blocks - 1; sl >= n; --sl) c->free_slots.push_back(sl);
  c->have_forest = true;
  c->have_data = false;
  c->have_flags = false;
  return upload_topo(c);
}

mrb_status mrb_load_blocks(mrb_ctx* c, const double* data, int on_device) {
  if (!c) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (!check_state(c, false)) return MRB_E_STATE;
  if (!data) return fail(c, MRB_E_ARG, "load_blocks: null data");
  const int n = (int)c->leaves.size();
  const size_t bytes = (size_t)n * c->bsz * sizeof(double);
  mrb_status s;
  const double* src = data;
  if (!on_device) {
    if ((s = ensure_scratch(c, bytes))) return s;
    HIPCHK(c, hipMemcpyAsync(c->dscratch, data, bytes, hipMemcpyHostToDevice, c->stream));
    src = c->dscratch;
  }
  std::vector<int> slots(n);
  for (int i = 0; i < n; ++i) slots[i] = c->leaves[i].slot;
  if ((s = stage_upload(c, c->st_slots, slots.data(), n * sizeof(int), c->dslots))) return s;
  HIPCHK(c, launch_scatter(src, c->dslots, n, c->bsz, c->u, c->stream));
  if (!on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
  c->have_data = true;
  c->have_flags = false;
  return MRB_OK;
}

mrb_status mrb_refine_all(mrb_ctx* c) {
  if (!c) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (!check_state(c, true)) return MRB_E_STATE;
  return do_refine_all(c);
}

mrb_status mrb_rk4(mrb_ctx* c, double t, double dt) {
  if (!c) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (!check_state(c, true)) return MRB_E_STATE;
  if (!(dt > 0.0) || !std::isfinite(t)) return fail(c, MRB_E_ARG, "rk4: dt must be positive");
  c->have_flags = false;
  return do_rk4(c, t, dt);
}

mrb_status mrb_mr_pass(mrb_ctx* c, int8_t* flags, double* maxd) {
  if (!c) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (!check_state(c, true)) return MRB_E_STATE;
  mrb_status s = do_mr_pass(c);
  if (flags) std::memcpy(flags, c->last_flags.data(), c->last_flags.size());
  if (maxd) std::memcpy(maxd, c->last_maxd.data(), c->last_maxd.size() * sizeof(double));
  return s;
}

mrb_status mrb_mr_pass_noalloc(mrb_ctx* c, int8_t* flags, double* maxd) {
  if (!c) return MRB_E_ARG;
  if (!check_state(c, true)) return MRB_E_STATE;
  if (!c->scratch_dev) return fail(c, MRB_E_DEVICE, "mr_pass_noalloc: no scratch on this device: " + c->scratch_err);
  // works on whichever side holds the topology (no pull: that could allocate)
  const size_t n = nblk(c), nf = (size_t)c->cfg.nfields;
  const size_t acc_bytes = (n * nf * sizeof(unsigned long long) + 255) & ~(size_t)255;
  const size_t need = acc_bytes + n * sizeof(int);
  if (need > kScratchBytes)
    return fail(c, MRB_E_CAPACITY, "mr_pass_noalloc: " + std::to_string(n) + " blocks x " + std::to_string(nf) +
                                       " fields exceed the " + std::to_string(kScratchBytes) + "-byte scratch");
  // sub-tiled workgroups: the tuned analysis tiling when it is sub-tiled, else 2 per axis
  int va[8];
  const int na = aux_variants(c->shape, 0, va, 8);
  int ns = c->nsub_mr > 1 ? c->nsub_mr : 2;
  bool compiled = false;
  for (int i = 0; i < na; ++i) compiled = compiled || va[i] == ns;
  if (!compiled) return fail(c, MRB_E_ARG, "mr_pass_noalloc: no sub-tiled analysis kernel for this shape");
  // partial maxima and completion counters start at zero (the previous call may have
  // left other contents; a fill kernel, so the call can be captured)
  char* base = (char*)c->scratch_dev;
  HIPCHK(c, launch_zero(base, need, c->stream));
  MrArgs a = mr_args(c);
  a.acc = (unsigned long long*)base;
  a.done = (int*)(base + acc_bytes);
  long work = (long)n;
  for (int q = 0; q < c->cfg.dim; ++q) work *= ns;
  HIPCHK(c, launch_mr(c->shape, ns, 256, grid_for(c, work), a, c->stream));
  mrb_status r = mr_readback(c);
  c->dev.have_flags = false;   // the newest analysis is the host's copy
  if (flags) std::memcpy(flags, c->last_flags.data(), c->last_flags.size());
  if (maxd) std::memcpy(maxd, c->last_maxd.data(), c->last_maxd.size() * sizeof(double));
  return r;
}

mrb_status mrb_coarsen(mrb_ctx* c, const int8_t* flags, int* n_coarsened) {
  if (!c) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (!check_state(c, true)) return MRB_E_STATE;
  if (!flags) return fail(c, MRB_E_ARG, "coarsen: null flags");
  std::vector<int8_t> fl(flags, flags + c->leaves.size());
  return do_coarsen(c, fl.data(), n_coarsened);
}

mrb_status mrb_adapt(mrb_ctx* c, int* n_passes) {
  if (!c) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (!check_state(c, true)) return MRB_E_STATE;
  return do_adapt(c, n_passes);
}

mrb_status mrb_step(mrb_ctx* c, double t0, double dt, int nsteps) {
  if (!c) return MRB_E_ARG;
  if (!check_state(c, true)) return MRB_E_STATE;
  if (nsteps < 0 || !(dt > 0.0)) return fail(c, MRB_E_ARG, "step: bad dt or nsteps");
  constexpr size_t kGraphProbe = 10;
  for (int s = 0; s < nsteps; ++s) {
    mrb_status r;
    // planning on the device or on the host (the forest moves between them as needed)
    const bool on_dev = want_device(c);
    if (on_dev != c->dev.active && (r = on_dev ? dev_push(c) : dev_pull(c))) return r;
    if (on_dev) {
      if ((r = dev_refine_all(c))) return r;
      if ((r = do_rk4(c, t0 + s * dt, dt))) return r;
      if ((r = dev_adapt(c, nullptr))) return r;
      c->dev.steps++;
      c->n_steps++;
      continue;
    }
    bool probing = false;
    if (c->graph_mode == 2) {
      const size_t n0 = c->probe_us[0].size(), n1 = c->probe_us[1].size();
      if (n0 < kGraphProbe || n1 < kGraphProbe) {
        probing = true;
        c->use_graph = n1 <= n0;   // alternate, graph first
      }
    }
    const double w0 = probing ? now_us() : 0.0;
    if (graph_ok(c)) {
      if ((r = step_graph(c, t0 + s * dt, dt))) return r;
    } else {
      if (!probing && s + 1 < nsteps) {
        // forests that cycle through the one-launch step: queued steps (counted inside)
        int done = 0;
        if ((r = steps_cycled(c, t0 + s * dt, dt, nsteps - s, &done))) return r;
        if (done > 0) {
          s += done - 1;
          continue;
        }
      }
      const bool fold = refine_foldable(c);
      if ((r = do_refine_all(c, !fold))) return r;
      bool tiled = false;
      if ((r = rk4_adapt_tiled(c, t0 + s * dt, dt, &tiled, fold))) return r;
      if (fold && !tiled) return fail(c, MRB_E_STATE, "folded refinement was not launched");
      if (!tiled && (r = do_rk4(c, t0 + s * dt, dt))) return r;
      if (!tiled && (r = do_adapt(c, nullptr, false, false))) return r;
    }
    if (probing) {
      c->probe_us[c->use_graph ? 1 : 0].push_back(now_us() - w0);
      if (c->probe_us[0].size() >= kGraphProbe && c->probe_us[1].size() >= kGraphProbe) {
        auto med = [](std::vector<double> v) {
          std::sort(v.begin(), v.end());
          return v[v.size() / 2];
        };
        // the first graph step pays for the capture: medians ignore it
        c->use_graph = med(c->probe_us[1]) < med(c->probe_us[0]);
      }
    }
    c->n_steps++;
  }
  return MRB_OK;
}

mrb_status mrb_num_blocks(mrb_ctx* c, int* n) {
  if (!c || !n) return MRB_E_ARG;
  if (!check_state(c, false)) return MRB_E_STATE;
  *n = (int)nblk(c);
  return MRB_OK;
}

mrb_status mrb_read_forest(mrb_ctx* c, int8_t* level, int32_t* coords) {
  if (!c || !level || !coords) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (!check_state(c, false)) return MRB_E_STATE;
  const int d = c->cfg.dim;
  for (size_t i = 0; i < c->leaves.size(); ++i) {
    level[i] = (int8_t)c->leaves[i].level;
    for (int a = 0; a < d; ++a) coords[i * d + a] = c->leaves[i].c[a];
  }
  return MRB_OK;
}

mrb_status mrb_read_blocks(mrb_ctx* c, double* out, int on_device) {
  if (!c || !out) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (!check_state(c, true)) return MRB_E_STATE;
  const int n = (int)c->leaves.size();
  const size_t bytes = (size_t)n * c->bsz * sizeof(double);
  mrb_status s;
  double* dst = out;
  if (!on_device) {
    if ((s = ensure_scratch(c, bytes))) return s;
    dst = c->dscratch;
  }
  ReadArgs a{topo(c), c->u, dst, 0};
  HIPCHK(c, launch_read(c->shape, grid_for(c, n), a, c->stream));
  if (!on_device) HIPCHK(c, hipMemcpyAsync(out, dst, bytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MRB_OK;
}

mrb_status mrb_read_uniform(mrb_ctx* c, int level, double* out, int on_device) {
  if (!c || !out) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (!check_state(c, true)) return MRB_E_STATE;
  if (level < 1 || level > c->cfg.jmax)
    return fail(c, MRB_E_ARG, "read_uniform: level must be between 1 and jmax");
  size_t pts = 1;
  for (int a = 0; a < c->cfg.dim; ++a) pts *= (size_t)(1L << level) * (size_t)(c->cfg.bs - 1);
  const size_t bytes = pts * c->cfg.nfields * sizeof(double);
  mrb_status s;
  double* dst = out;
  if (!on_device) {
    if ((s = ensure_scratch(c, bytes))) return s;
    dst = c->dscratch;
  }
  if ((s = read_uniform_to(c, level, dst))) return s;
  if (!on_device) HIPCHK(c, hipMemcpyAsync(out, dst, bytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MRB_OK;
}

mrb_status mrb_get_flags(mrb_ctx* c, int8_t* flags, double* maxd) {
  if (!c || !flags) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (!c->have_flags) return fail(c, MRB_E_STATE, "no analysis on the current grid");
  std::memcpy(flags, c->last_flags.data(), c->last_flags.size());
  if (maxd) std::memcpy(maxd, c->last_maxd.data(), c->last_maxd.size() * sizeof(double));
  return MRB_OK;
}

mrb_status mrb_stats(mrb_ctx* c, char* json, int cap) {
  if (!c || !json || cap <= 0) return MRB_E_ARG;
  resolve_timing(c);
  std::string kern = "{";
  for (int k = 0; k < T_NKIND; ++k) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s\"%s\": {\"launches\": %ld, \"ms\": %.6f, \"bytes\": %.17g}", k ? ", " : "",
                  kKindName[k], c->t_launches[k], c->t_ms[k], c->t_bytes[k]);
    kern += buf;
  }
  kern += "}";
  int w = std::snprintf(json, cap,
                "{\"blocks\": %zu, \"steps\": %ld, \"rk4\": %ld, \"block_updates\": %ld, \"mr_passes\": %ld, "
                "\"families_coarsened\": %ld, \"blocks_refined\": %ld, \"free_slots\": %zu, \"grid\": %d, "
                "\"stage_tiles\": %d, \"stage_threads\": %d, \"stage_order\": \"%s\", \"analysis_threads\": %d, \"graph_launches\": %ld, \"graph_mode\": %d, \"graph_in_use\": %d, \"memo_hits\": %ld, \"spec_hits\": %ld, \"spec_misses\": %ld, \"queued_steps\": %ld, \"queued_taken_back\": %ld, \"sweep_launch\": \"%s\", \"rk4_tile_tiles\": %d, \"rk4_tile_tuned\": %d, \"rk4_tile_analysis\": [%d, %d], \"rk4_tile_refine\": [%d, %d, %d], \"rk4_tile_mothers\": [%d, %d], \"sweep_grid\": %d, \"topology\": \"%s\", \"topology_mode\": %d, \"device_topology\": {\"steps\": %ld, \"passes\": %ld, \"pushes\": %ld, \"pulls\": %ld}, \"host_us\": {\"refine_plan\": %.1f, "
                "\"coarsen_plan\": %.1f, \"upload\": %.1f, \"wait\": %.1f, \"graph_launch\": %.1f, \"plan_ordering\": %.1f, "
                "\"plan_entries\": %.1f, \"plan_entries_per_block\": %.1f, \"plan_fixed_point\": %.1f}, "
                "\"tune_ms\": {%s}, \"kernels\": %s}",
                nblk(c), c->n_steps, c->n_rk4, c->n_block_updates, c->n_mr, c->n_fam, c->n_refined,
                c->dev.active ? (size_t)c->dev.top : c->free_slots.size(), c->grid, c->have_forest && c->cfg.form == MRB_FORM_FUSED ? pick_nsub(c) : 1,
                c->have_forest && c->cfg.form == MRB_FORM_FUSED ? pick_tpb(c, pick_nsub(c)) : 256,
                c->order ? "level-sorted" : "forest", c->tpb_mr,
                c->n_graph_launches, c->graph_mode, c->use_graph ? 1 : 0, c->memo_hits, c->spec_hits, c->spec_misses, c->n_queued, c->n_taken_back,
                c->have_forest && rk4t_pick(c) > 0 ? "rk4_tile" : (sweep_in_one(c) ? "one" : "four"), c->rk4t_nsub,
                c->rk4t_tuned ? 1 : 0, c->ana_nsub, c->ana_tpb, c->ref_fold, c->ref_nsub, c->ref_tpb, c->ma_nsub, c->ma_tpb, c->sweep_grid, c->dev.active ? "device" : "host",
                c->dev.mode, c->dev.steps, c->dev.passes, c->dev.pushes, c->dev.pulls, c->hus_refine_plan, c->hus_coarsen_plan, c->hus_upload, c->hus_wait,
                c->hus_launch, c->hus_index, c->hus_desc, c->hus_desc_par, c->hus_fixed, c->tune_log.c_str(), kern.c_str());
  if (w < 0 || w >= cap) return fail(c, MRB_E_ARG, "stats: buffer too small");
  return MRB_OK;
}

mrb_status mrb_tune(mrb_ctx* c, int nsub, int reps, double dt, int* chosen) {
  if (!c) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  int v[8];
  const int nv = stage_variants(c->shape, c->cfg.precision, v, 8);
  if (nsub > 0) {
    bool ok = false;
    for (int i = 0; i < nv; ++i) ok = ok || v[i] == nsub;
    if (!ok) return fail(c, MRB_E_ARG, "tune: tiling not compiled for this shape and precision");
    c->nsub = nsub;
    c->tpb = 256;
    int tv[8];
    const int nt = rk4t_variants(c->shape, c->cfg.precision, tv, 8);
    for (int i = 0; i < nt; ++i)
      if (tv[i] == nsub) c->rk4t_nsub = nsub;
    c->ana_nsub = 0;
    c->ana_tpb = 256;
    c->ref_fold = 1;
    c->ref_nsub = 0;
    c->ref_tpb = 256;
    c->ma_nsub = 0;
    c->ma_tpb = 256;
    c->tpb_mr = 256;
    if (reps < 0) {
      // -reps threads per workgroup for the stage sweep, the whole-block analysis and the
      // tile step's folded forms, each where that form is compiled
      const int tpb = -reps;
      int tp[8];
      const int ntp = stage_threads(c->shape, c->cfg.precision, nsub, tp, 8);
      bool any = false;
      for (int i = 0; i < ntp; ++i)
        if (tp[i] == tpb) {
          c->tpb = tpb;
          any = true;
        }
      const int nmt = mr_threads(c->shape, 1, tp, 8);
      for (int i = 1; i < nmt; ++i)
        if (tp[i] == tpb) {
          c->tpb_mr = tpb;
          any = true;
        }
      if (c->rk4t_nsub == nsub && (tpb == 256 || ((tpb == 512 || tpb == 1024) && nsub <= 2))) {
        c->ana_nsub = c->ref_nsub = c->ma_nsub = nsub;
        c->ana_tpb = c->ref_tpb = c->ma_tpb = tpb;
        any = true;
      }
      if (!any) return fail(c, MRB_E_ARG, "tune: no form compiled with that tiling and workgroup size");
    }
  } else if (reps > 0) {
    if (!check_state(c, true)) return MRB_E_STATE;
    if (!(dt > 0.0)) return fail(c, MRB_E_ARG, "tune: dt must be positive");
    if (c->cfg.form != MRB_FORM_FUSED) return fail(c, MRB_E_ARG, "tune: only the fused form has tilings");
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    c->tune_log.clear();
    const bool was_timing = c->timing;
    c->timing = false;
    auto done = [&](mrb_status r) {
      c->have_flags = false;
      c->timing = was_timing;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return r;
    };
    // stage tilings (sub-tiles per axis x threads per workgroup) x processing order
    // (forest/Morton, level-sorted); as below, the fastest of several rounds counts
    constexpr int kRounds = 5;
    struct Cand { int nsub, tpb, order; float ms; };
    std::vector<Cand> cand;
    for (int i = 0; i < nv; ++i) {
      int tv[4];
      const int nt = stage_threads(c->shape, c->cfg.precision, v[i], tv, 4);
      for (int j = 0; j < nt; ++j)
        for (int o = 0; o < 2; ++o) cand.push_back(Cand{v[i], tv[j], o, 1e30f});
    }
    for (int round = 0; round < kRounds; ++round)
      for (Cand& k : cand) {
        c->nsub = k.nsub;
        c->tpb = k.tpb;
        c->order = k.order;
        mrb_status r = sweep(c, 0.0, dt);  // warm-up
        if (r) return done(r);
        if (hipEventRecord(e0, c->stream) != hipSuccess) return done(fail(c, MRB_E_DEVICE, "tune: event"));
        for (int q = 0; q < reps; ++q)
          if ((r = sweep(c, 0.0, dt))) return done(r);
        float ms = 0.f;
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
          return done(fail(c, MRB_E_DEVICE, "tune: event"));
        k.ms = std::min(k.ms, ms / reps);
      }
    size_t bi = 0;
    for (size_t i = 0; i < cand.size(); ++i) {
      // keys: sub-tiles per axis, "t<threads>" unless 256, "L" for the level-sorted order
      char buf[64], tp[16] = "";
      if (cand[i].tpb != 256) std::snprintf(tp, sizeof tp, "t%d", cand[i].tpb);
      std::snprintf(buf, sizeof buf, "%s\"%d%s%s\": %.4f", i ? ", " : "", cand[i].nsub, tp, cand[i].order ? "L" : "",
                    cand[i].ms);
      c->tune_log += buf;
      if (cand[i].ms < cand[bi].ms) bi = i;
    }
    c->nsub = cand[bi].nsub;
    c->tpb = cand[bi].tpb;
    c->order = cand[bi].order;
    // one launch with grid barriers against four launches, on the chosen tiling
    {
      const int mode0 = c->sweep_mode;
      float best_m[2] = {1e30f, 1e30f};
      bool one_ok = true;
      for (int round = 0; round < kRounds && one_ok; ++round)
        for (int m = 0; m < 2 && one_ok; ++m) {
          c->sweep_mode = m;
          mrb_status r = MRB_OK;
          for (int k = 0; k < reps + 1 && !r; ++k) {   // the first is a warm-up
            if (k == 1 && hipEventRecord(e0, c->stream) != hipSuccess) r = MRB_E_DEVICE;
            if (!r) r = sweep(c, 0.0, dt);
          }
          float ms = 0.f;
          if (!r && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                     hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            r = MRB_E_DEVICE;
          if (!r) r = check_barrier(c);
          if (r) {
            if (m == 0) { c->sweep_mode = mode0; return done(r); }
            // the one-launch form is not available here (e.g. the cooperative launch
            // was refused): keep four launches
            (void)hipGetLastError();
            (void)hipStreamSynchronize(c->stream);
            one_ok = false;
            break;
          }
          best_m[m] = std::min(best_m[m], ms / reps);
        }
      c->sweep_mode = mode0;
      c->sweep_one_tuned = one_ok && best_m[1] < best_m[0];
      char buf[96];
      std::snprintf(buf, sizeof buf, ", \"sweep\": {\"four\": %.4f, \"one\": %.4f}", best_m[0],
                    one_ok ? best_m[1] : -1.0f);
      c->tune_log += buf;
    }
    // the overlapped-tile RK4 step (forests on one level; every tiling compiled for the
    // shape) against the stage launches chosen above
    c->rk4t_tuned = false;
    {
      int tv[8];
      const int nt = rk4t_variants(c->shape, c->cfg.precision, tv, 8);
      if (nt > 0 && one_level(c)) {
        const int mode0 = c->sweep_mode, nsub0 = c->rk4t_nsub;
        float best_t[9];
        for (int i = 0; i <= nt; ++i) best_t[i] = 1e30f;
        mrb_status r = MRB_OK;
        for (int round = 0; round < kRounds && !r; ++round)
          for (int i = 0; i <= nt && !r; ++i) {
            if (i < nt) {
              c->sweep_mode = 3;
              c->rk4t_nsub = tv[i];
            } else {
              c->sweep_mode = mode0 == 3 ? 2 : mode0;   // the stage launches
            }
            for (int k = 0; k < reps + 1 && !r; ++k) {   // the first is a warm-up
              if (k == 1 && hipEventRecord(e0, c->stream) != hipSuccess) r = MRB_E_DEVICE;
              if (!r) r = sweep(c, 0.0, dt);
            }
            float ms = 0.f;
            if (!r && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                       hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
              r = fail(c, MRB_E_DEVICE, "tune: event");
            if (!r) r = check_barrier(c);
            if (!r) best_t[i] = std::min(best_t[i], ms / reps);
          }
        c->sweep_mode = mode0;
        if (r) {
          c->rk4t_nsub = nsub0;
          return done(r);
        }
        int bi = 0;
        c->tune_log += ", \"rk4_tile\": {";
        for (int i = 0; i < nt; ++i) {
          char buf[48];
          std::snprintf(buf, sizeof buf, "\"%d\": %.4f, ", tv[i], best_t[i]);
          c->tune_log += buf;
          if (best_t[i] < best_t[bi]) bi = i;
        }
        char buf[48];
        std::snprintf(buf, sizeof buf, "\"stages\": %.4f}", best_t[nt]);
        c->tune_log += buf;
        c->rk4t_nsub = tv[bi];
        c->rk4t_tuned = best_t[bi] < best_t[nt];
        // the first analysis folded into the tile launch (tilings x threads) against
        // the tile launch followed by an analysis launch
        c->ana_nsub = -1;
        struct AC { int nsub, tpb; float ms; };
        std::vector<AC> ac;
        if (c->rk4t_tuned) {
          for (int i = 0; i < nt; ++i)
            for (int tp : {256, 512, 1024})
              if (tp == 256 || tv[i] <= 2) ac.push_back(AC{tv[i], tp, 1e30f});
          float pair = 1e30f;
          Rk4tArgs ra = rk4t_args(c, 0.0, dt);
          rk4t_analysis_args(c, ra, nullptr);
          for (int round = 0; round < kRounds && !r; ++round)
            for (size_t i = 0; i <= ac.size() && !r; ++i) {
              for (int k = 0; k < reps + 1 && !r; ++k) {   // the first is a warm-up
                if (k == 1 && hipEventRecord(e0, c->stream) != hipSuccess) r = MRB_E_DEVICE;
                if (r) break;
                if (i < ac.size()) {
                  r = launch_tiled(c, ac[i].nsub, ra, true, ac[i].tpb);
                } else {
                  r = launch_tiled(c, c->rk4t_nsub, ra, false);
                  c->flag_set = 0;
                  if (!r) r = launch_mr_kernel(c, false);
                }
              }
              float ms = 0.f;
              if (!r && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                r = fail(c, MRB_E_DEVICE, "tune: event");
              if (r) break;
              if (i < ac.size()) ac[i].ms = std::min(ac[i].ms, ms / reps);
              else pair = std::min(pair, ms / reps);
            }
          if (r) return done(r);
          size_t bj = 0;
          c->tune_log += ", \"rk4_tile_analysis\": {";
          for (size_t i = 0; i < ac.size(); ++i) {
            char buf[48];
            std::snprintf(buf, sizeof buf, "\"%d%s\": %.4f, ", ac[i].nsub,
                          ac[i].tpb == 256 ? "" : (ac[i].tpb == 512 ? "t512" : "t1024"), ac[i].ms);
            c->tune_log += buf;
            if (ac[i].ms < ac[bj].ms) bj = i;
          }
          char buf[48];
          std::snprintf(buf, sizeof buf, "\"separate\": %.4f}", pair);
          c->tune_log += buf;
          if (ac[bj].ms < pair) {
            c->ana_nsub = ac[bj].nsub;
            c->ana_tpb = ac[bj].tpb;
          }
        }
        // the refinement folded in as well, right after a refine-all of a forest on one
        // level (its plan is the uploaded one and the parents' data is intact): one
        // launch per tiling and thread count against the refinement launch followed by
        // the chosen tile launch
        c->ref_fold = 1;
        c->ref_nsub = 0;
        c->ref_tpb = 256;
        if (c->ana_nsub > 0 && (long)c->pending_ref * (1 << c->cfg.dim) == (long)nblk(c)) {
          std::vector<float> best_f(ac.size() + 1, 1e30f);
          Rk4tArgs ra = rk4t_args(c, 0.0, dt);
          rk4t_analysis_args(c, ra, nullptr);
          for (int round = 0; round < kRounds && !r; ++round)
            for (size_t m = 0; m <= ac.size() && !r; ++m) {
              for (int k = 0; k < reps + 1 && !r; ++k) {   // the first is a warm-up
                if (k == 1 && hipEventRecord(e0, c->stream) != hipSuccess) r = MRB_E_DEVICE;
                if (r) break;
                if (m < ac.size()) {
                  r = launch_tiled(c, ac[m].nsub, ra, true, ac[m].tpb, true);
                } else {
                  r = launch_refine_kernel(c, c->pending_ref, false);
                  if (!r) r = launch_tiled(c, c->ana_nsub, ra, true, c->ana_tpb);
                }
              }
              float ms = 0.f;
              if (!r && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                r = fail(c, MRB_E_DEVICE, "tune: event");
              if (!r) best_f[m] = std::min(best_f[m], ms / reps);
            }
          if (r) return done(r);
          size_t bf = 0;
          c->tune_log += ", \"rk4_tile_refine\": {";
          for (size_t i = 0; i < ac.size(); ++i) {
            char buf[48];
            std::snprintf(buf, sizeof buf, "\"%d%s\": %.4f, ", ac[i].nsub,
                          ac[i].tpb == 256 ? "" : (ac[i].tpb == 512 ? "t512" : "t1024"), best_f[i]);
            c->tune_log += buf;
            if (best_f[i] < best_f[bf]) bf = i;
          }
          char buf[48];
          std::snprintf(buf, sizeof buf, "\"separate\": %.4f}", best_f[ac.size()]);
          c->tune_log += buf;
          c->ref_fold = best_f[bf] < best_f[ac.size()] ? 1 : 0;
          c->ref_nsub = ac[bf].nsub;
          c->ref_tpb = ac[bf].tpb;
          // with the second analysis of a coarsening that merges every block folded in
          // too: timed with a map that sends each block's mother nodes into its own
          // slot of u_new (scratch during tuning) and its child index from forest order
          c->ma_nsub = 0;
          c->ma_tpb = 256;
          if (c->dmq) {
            const int n = (int)nblk(c), nch = 1 << c->cfg.dim;
            std::vector<int> hm(n);
            for (int b = 0; b < n; ++b) hm[b] = c->hblk[b].slot * 8 + b % nch;
            int* dm = nullptr;
            if (hipMalloc((void**)&dm, n * sizeof(int)) != hipSuccess) return done(fail(c, MRB_E_DEVICE, "tune: map"));
            if (hipMemcpy(dm, hm.data(), n * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
              (void)hipFree(dm);
              return done(fail(c, MRB_E_DEVICE, "tune: map"));
            }
            std::vector<float> best_m(ac.size(), 1e30f);
            Rk4tArgs rm = ra;
            rm.smap = dm;
            rm.mq = c->dmq;
            for (int round = 0; round < kRounds && !r; ++round)
              for (size_t m = 0; m < ac.size() && !r; ++m) {
                for (int k = 0; k < reps + 1 && !r; ++k) {
                  if (k == 1 && hipEventRecord(e0, c->stream) != hipSuccess) r = MRB_E_DEVICE;
                  if (!r) r = launch_tiled(c, ac[m].nsub, rm, true, ac[m].tpb, true, true);
                }
                float ms = 0.f;
                if (!r && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                  r = fail(c, MRB_E_DEVICE, "tune: event");
                if (!r) best_m[m] = std::min(best_m[m], ms / reps);
              }
            (void)hipFree(dm);
            if (r) return done(r);
            size_t bm = 0;
            c->tune_log += ", \"rk4_tile_mothers\": {";
            for (size_t i = 0; i < ac.size(); ++i) {
              char buf[48];
              std::snprintf(buf, sizeof buf, "%s\"%d%s\": %.4f", i ? ", " : "", ac[i].nsub,
                            ac[i].tpb == 256 ? "" : (ac[i].tpb == 512 ? "t512" : "t1024"), best_m[i]);
              c->tune_log += buf;
              if (best_m[i] < best_m[bm]) bm = i;
            }
            c->tune_log += "}";
            c->ma_nsub = ac[bm].nsub;
            c->ma_tpb = ac[bm].tpb;
          }
        }
      }
    }
    // analysis and refinement tilings: several rounds over the candidates, the fastest
    // round of each counts (single launches of these kernels are a few microseconds on
    // small grids, where one round is at the mercy of noise)
    int va[8];
    const int na = aux_variants(c->shape, 0, va, 8);
    auto time_variants = [&](const char* name, int* choice, auto&& run) -> mrb_status {
      float best_v[8];
      for (int i = 0; i < na; ++i) best_v[i] = 1e30f;
      for (int round = 0; round < kRounds; ++round)
        for (int i = 0; i < na; ++i) {
          *choice = va[i];
          mrb_status r = run(va[i], 1);  // warm-up (also loads the variant)
          if (r) return r;
          if (hipEventRecord(e0, c->stream) != hipSuccess) return fail(c, MRB_E_DEVICE, "tune: event");
          if ((r = run(va[i], reps))) return r;
          float ms = 0.f;
          if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return fail(c, MRB_E_DEVICE, "tune: event");
          best_v[i] = std::min(best_v[i], ms / reps);
        }
      int bi = 0;
      c->tune_log += std::string(", \"") + name + "\": {";
      for (int i = 0; i < na; ++i) {
        char buf[64];
        std::snprintf(buf, sizeof buf, "%s\"%d\": %.4f", i ? ", " : "", va[i], best_v[i]);
        c->tune_log += buf;
        if (best_v[i] < best_v[bi]) bi = i;
      }
      c->tune_log += "}";
      *choice = va[bi];
      return MRB_OK;
    };
    // an analysis pass only synchronises redundant nodes (idempotent) and rewrites
    // flags and maxima
    {
      mrb_status r = do_mr_pass(c);
      if (r && r != MRB_E_NONFINITE) return done(r);
    }
    mrb_status tr = time_variants("mr", &c->nsub_mr, [&](int v, int k) -> mrb_status {
      MrArgs a = mr_args(c);
      const int n = (int)c->hblk.size();
      long work = n;
      for (int q = 0; q < c->cfg.dim; ++q) work *= v;
      for (int j = 0; j < k; ++j) HIPCHK(c, launch_mr(c->shape, v, 256, grid_for(c, work), a, c->stream));
      return MRB_OK;
    });
    if (tr) return done(tr);
    // whole blocks: the analysis with larger workgroups where compiled
    c->tpb_mr = 256;
    if (c->nsub_mr == 1) {
      int tp[4];
      const int nt = mr_threads(c->shape, 1, tp, 4);
      if (nt > 1) {
        float best[4] = {1e30f, 1e30f, 1e30f, 1e30f};
        MrArgs a = mr_args(c);
        const long work = (long)c->hblk.size();
        for (int round = 0; round < kRounds; ++round)
          for (int i = 0; i < nt; ++i) {
            HIPCHK(c, launch_mr(c->shape, 1, tp[i], grid_for(c, work), a, c->stream));   // warm-up
            HIPCHK(c, hipEventRecord(e0, c->stream));
            for (int j = 0; j < reps; ++j) HIPCHK(c, launch_mr(c->shape, 1, tp[i], grid_for(c, work), a, c->stream));
            float ms = 0.f;
            if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
              return done(fail(c, MRB_E_DEVICE, "tune: event"));
            best[i] = std::min(best[i], ms / reps);
          }
        int bi = 0;
        c->tune_log += ", \"mr_threads\": {";
        for (int i = 0; i < nt; ++i) {
          char buf[48];
          std::snprintf(buf, sizeof buf, "%s\"%d\": %.4f", i ? ", " : "", tp[i], best[i]);
          c->tune_log += buf;
          if (best[i] < best[bi]) bi = i;
        }
        c->tune_log += "}";
        c->tpb_mr = tp[bi];
      }
    }
    // refinement, while the last refinement plan is still the uploaded one: re-running
    // it rewrites the same children from the untouched parents
    if (c->pending_ref > 0) {
      tr = time_variants("refine", &c->nsub_ref, [&](int, int k) -> mrb_status {
        for (int j = 0; j < k; ++j) {
          mrb_status r = launch_refine_kernel(c, c->pending_ref, false);
          if (r) return r;
        }
        return MRB_OK;
      });
      if (tr) return done(tr);
    }
    (void)done(MRB_OK);
  } else {
    c->nsub = 0;
    c->tpb = 256;
    c->nsub_mr = -1;
    c->tpb_mr = 256;
    c->nsub_ref = 0;
    c->order = 0;
    c->rk4t_nsub = 0;
    c->rk4t_tuned = false;
    c->ana_nsub = 0;
    c->ana_tpb = 256;
    c->ref_fold = 1;
    c->ref_nsub = 0;
    c->ref_tpb = 256;
    c->ma_nsub = 0;
    c->ma_tpb = 256;
  }
  if (chosen) *chosen = c->cfg.form == MRB_FORM_FUSED ? pick_nsub(c) : 1;
  return MRB_OK;
}

// ---------------------------------------------------------------------------
// learned predictor
// ---------------------------------------------------------------------------
namespace {

mrb_status mlp_ready(mrb_ctx* c) {
  if (!c->mp) return fail(c, MRB_E_STATE, "predictor not initialised (mrb_mlp_init)");
  return MRB_OK;
}

mrb_status mlp_workspace(mrb_ctx* c, int n) {
  if (n <= c->mlp_cap) return MRB_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float** fl[] = {&c->mx, &c->mxn, &c->mz1, &c->ma1, &c->mz2, &c->ma2, &c->mlog, &c->mloss, &c->mdl, &c->mdz1,
                  &c->mdz2, &c->mpmax};
  for (float** p : fl)
    if (*p) { (void)hipFree(*p); *p = nullptr; }
  if (c->my) { (void)hipFree(c->my); c->my = nullptr; }
  if (c->mpred) { (void)hipFree(c->mpred); c->mpred = nullptr; }
  const size_t N = (size_t)n;
  HIPCHK(c, hipMalloc(&c->mx, N * c->mlp_nin * 4));
  HIPCHK(c, hipMalloc(&c->mxn, N * c->mlp_nin * 4));
  HIPCHK(c, hipMalloc(&c->mz1, N * 64 * 4));
  HIPCHK(c, hipMalloc(&c->ma1, N * 64 * 4));
  HIPCHK(c, hipMalloc(&c->mz2, N * 64 * 4));
  HIPCHK(c, hipMalloc(&c->ma2, N * 64 * 4));
  HIPCHK(c, hipMalloc(&c->mlog, N * 3 * 4));
  HIPCHK(c, hipMalloc(&c->mloss, N * 4));
  HIPCHK(c, hipMalloc(&c->mdl, N * 3 * 4));
  HIPCHK(c, hipMalloc(&c->mdz1, N * 64 * 4));
  HIPCHK(c, hipMalloc(&c->mdz2, N * 64 * 4));
  HIPCHK(c, hipMalloc(&c->mpmax, N * 4));
  HIPCHK(c, hipMalloc(&c->my, N));
  HIPCHK(c, hipMalloc(&c->mpred, N));
  c->mlp_cap = n;
  return MRB_OK;
}

MlpArgs mlp_args(mrb_ctx* c, int off, int n) {
  MlpArgs a;
  std::memset(&a, 0, sizeof a);
  a.p = c->mp;
  a.nin = c->mlp_nin;
  a.n = n;
  const size_t o = (size_t)off;
  a.x = c->mx + o * c->mlp_nin;
  a.mean = c->mnorm;
  a.std = c->mnorm + 4;
  a.xn = c->mxn + o * c->mlp_nin;
  a.z1 = c->mz1 + o * 64;
  a.a1 = c->ma1 + o * 64;
  a.z2 = c->mz2 + o * 64;
  a.a2 = c->ma2 + o * 64;
  a.logits = c->mlog + o * 3;
  a.y = c->my + o;
  a.classw = c->mcw;
  a.loss = c->mloss + o;
  a.dl = c->mdl + o * 3;
  a.dz1 = c->mdz1 + o * 64;
  a.dz2 = c->mdz2 + o * 64;
  a.g = c->mgrad;
  return a;
}

// features of the current forest into the workspace (device)
mrb_status mlp_features_dev(mrb_ctx* c) {
  const int n = (int)c->hblk.size();
  mrb_status r = mlp_workspace(c, n);
  if (r) return r;
  MlpPoolArgs a{topo(c), c->u, c->cfg.nfields, c->mx};
  HIPCHK(c, launch_pool(c->cfg.bs, grid_for(c, n), a, c->stream));
  return MRB_OK;
}

double batch_inv_wsum(const int8_t* y, int n, const float* cw) {
  double W = 0.0;
  for (int i = 0; i < n; ++i) W += cw[y[i]];
  return W > 0.0 ? 1.0 / W : 0.0;
}

}  // namespace

mrb_status mrb_mlp_init(mrb_ctx* c, int nin, const float* params, const float* mean, const float* std) {
  if (!c) return MRB_E_ARG;
  if (c->cfg.dim != 2 || (c->cfg.bs != 17 && c->cfg.bs != 33))
    return fail(c, MRB_E_ARG, "mlp: 2D blocks of 17 or 33 points only");
  if (nin != c->cfg.nfields * 64) return fail(c, MRB_E_ARG, "mlp: nin must be 64 per field");
  if (!params || !mean || !std) return fail(c, MRB_E_ARG, "mlp: null parameters or normalisation");
  for (int f = 0; f < c->cfg.nfields; ++f)
    if (!(std[f] > 0.0f)) return fail(c, MRB_E_ARG, "mlp: std must be positive");
  const int np = mlp_param_count(nin);
  if (!c->mp || c->mlp_np != np) {
    float** bufs[] = {&c->mp, &c->mgrad, &c->mm, &c->mv};
    for (float** b : bufs) {
      if (*b) (void)hipFree(*b);
      *b = nullptr;
      HIPCHK(c, hipMalloc(b, (size_t)np * 4));
    }
    if (!c->mnorm) HIPCHK(c, hipMalloc(&c->mnorm, 8 * 4));
    if (!c->mcw) HIPCHK(c, hipMalloc(&c->mcw, 4 * 4));
  }
  c->mlp_nin = nin;
  c->mlp_np = np;
  c->mlp_t = 0;
  float norm[8] = {0, 0, 0, 0, 1, 1, 1, 1};
  for (int f = 0; f < c->cfg.nfields; ++f) {
    norm[f] = mean[f];
    norm[4 + f] = std[f];
  }
  HIPCHK(c, hipMemcpyAsync(c->mp, params, (size_t)np * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->mnorm, norm, sizeof norm, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemsetAsync(c->mm, 0, (size_t)np * 4, c->stream));
  HIPCHK(c, hipMemsetAsync(c->mv, 0, (size_t)np * 4, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MRB_OK;
}

mrb_status mrb_mlp_get_params(mrb_ctx* c, float* params) {
  if (!c || !params) return MRB_E_ARG;
  if (mlp_ready(c)) return MRB_E_STATE;
  HIPCHK(c, hipMemcpyAsync(params, c->mp, (size_t)c->mlp_np * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MRB_OK;
}

mrb_status mrb_mlp_features(mrb_ctx* c, float* feat) {
  if (!c || !feat) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (!check_state(c, true)) return MRB_E_STATE;
  if (c->cfg.dim != 2 || (c->cfg.bs != 17 && c->cfg.bs != 33)) return fail(c, MRB_E_ARG, "features: 2D only");
  if (!c->mlp_nin) c->mlp_nin = c->cfg.nfields * 64;
  mrb_status r = mlp_features_dev(c);
  if (r) return r;
  HIPCHK(c, hipMemcpyAsync(feat, c->mx, c->hblk.size() * c->cfg.nfields * 64 * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MRB_OK;
}

mrb_status mrb_mlp_forward(mrb_ctx* c, const float* x, int n, float* logits) {
  if (!c || !x || !logits || n <= 0) return MRB_E_ARG;
  if (mlp_ready(c)) return MRB_E_STATE;
  mrb_status r = mlp_workspace(c, n);
  if (r) return r;
  HIPCHK(c, hipMemcpyAsync(c->mx, x, (size_t)n * c->mlp_nin * 4, hipMemcpyHostToDevice, c->stream));
  MlpArgs a = mlp_args(c, 0, n);
  HIPCHK(c, launch_mlp_forward(a, c->stream));
  HIPCHK(c, hipMemcpyAsync(logits, c->mlog, (size_t)n * 3 * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MRB_OK;
}

mrb_status mrb_mlp_grad(mrb_ctx* c, const float* x, const int8_t* y, const float* classw, int n, float* grads,
                        float* loss) {
  if (!c || !x || !y || !classw || n <= 0) return MRB_E_ARG;
  if (mlp_ready(c)) return MRB_E_STATE;
  for (int i = 0; i < n; ++i)
    if (y[i] < 0 || y[i] > 2) return fail(c, MRB_E_ARG, "mlp: labels must be 0, 1 or 2");
  mrb_status r = mlp_workspace(c, n);
  if (r) return r;
  HIPCHK(c, hipMemcpyAsync(c->mx, x, (size_t)n * c->mlp_nin * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->my, y, (size_t)n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->mcw, classw, 3 * 4, hipMemcpyHostToDevice, c->stream));
  MlpArgs a = mlp_args(c, 0, n);
  a.inv_wsum = (float)batch_inv_wsum(y, n, classw);
  HIPCHK(c, launch_mlp_forward(a, c->stream));
  HIPCHK(c, launch_mlp_backward(a, c->stream));
  std::vector<float> ls(n);
  if (grads) HIPCHK(c, hipMemcpyAsync(grads, c->mgrad, (size_t)c->mlp_np * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(ls.data(), c->mloss, (size_t)n * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (loss) {
    double s = 0.0;
    for (float v : ls) s += v;
    *loss = (float)s;
  }
  return MRB_OK;
}

mrb_status mrb_mlp_train(mrb_ctx* c, const float* x, const int8_t* y, const float* classw, int n, int batch, float lr,
                         float* mean_loss) {
  if (!c || !x || !y || !classw || n <= 0 || batch <= 0 || !(lr > 0.0f)) return MRB_E_ARG;
  if (mlp_ready(c)) return MRB_E_STATE;
  for (int i = 0; i < n; ++i)
    if (y[i] < 0 || y[i] > 2) return fail(c, MRB_E_ARG, "mlp: labels must be 0, 1 or 2");
  mrb_status r = mlp_workspace(c, n);
  if (r) return r;
  HIPCHK(c, hipMemcpyAsync(c->mx, x, (size_t)n * c->mlp_nin * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->my, y, (size_t)n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->mcw, classw, 3 * 4, hipMemcpyHostToDevice, c->stream));
  const double b1 = 0.9, b2 = 0.999;
  int nb = 0;
  for (int off = 0; off < n; off += batch, ++nb) {
    const int m = std::min(batch, n - off);
    MlpArgs a = mlp_args(c, off, m);
    a.inv_wsum = (float)batch_inv_wsum(y + off, m, classw);
    HIPCHK(c, launch_mlp_forward(a, c->stream));
    HIPCHK(c, launch_mlp_backward(a, c->stream));
    c->mlp_t++;
    MlpAdamArgs ad{c->mp, c->mgrad, c->mm, c->mv, c->mlp_np, lr, (float)b1, (float)b2, 1e-8f,
                   (float)(1.0 - std::pow(b1, c->mlp_t)), (float)(1.0 - std::pow(b2, c->mlp_t))};
    HIPCHK(c, launch_adam(ad, c->stream));
  }
  std::vector<float> ls(n);
  HIPCHK(c, hipMemcpyAsync(ls.data(), c->mloss, (size_t)n * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (mean_loss) {
    double s = 0.0;
    for (float v : ls) s += v;
    *mean_loss = (float)(s / nb);
  }
  return MRB_OK;
}

mrb_status mrb_mlp_predict(mrb_ctx* c, int8_t* pred, float* prob) {
  if (!c || !pred) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (!check_state(c, true)) return MRB_E_STATE;
  if (mlp_ready(c)) return MRB_E_STATE;
  const int n = (int)c->hblk.size();
  mrb_status r = mlp_features_dev(c);
  if (r) return r;
  MlpArgs a = mlp_args(c, 0, n);
  HIPCHK(c, launch_mlp_forward(a, c->stream));
  HIPCHK(c, launch_pred(c->mlog, n, c->mpred, c->mpmax, c->stream));
  HIPCHK(c, hipMemcpyAsync(pred, c->mpred, (size_t)n, hipMemcpyDeviceToHost, c->stream));
  if (prob) HIPCHK(c, hipMemcpyAsync(prob, c->mpmax, (size_t)n * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MRB_OK;
}

}  // extern "C"

namespace {
// marked blocks plus every coarser leaf that must refine with them to keep the grid graded
std::vector<int> graded_closure(mrb_ctx* c, const int8_t* mask) {
  const int n = (int)c->leaves.size();
  std::vector<char> mk(n, 0);
  std::unordered_map<int, int> by_slot;
  by_slot.reserve(n * 2);
  for (int i = 0; i < n; ++i) by_slot[c->leaves[i].slot] = i;
  std::vector<int> work;
  for (int i = 0; i < n; ++i)
    if (mask[i] && c->leaves[i].level < c->cfg.jmax) { mk[i] = 1; work.push_back(i); }
  while (!work.empty()) {
    const int i = work.back();
    work.pop_back();
    const BlockDesc& B = c->hblk[i];
    for (int e = B.nb_begin; e < B.nb_begin + B.n_ent; ++e) {
      const NbEntry& E = c->hnb[e];
      if (E.dl >= 0) continue;
      const int j = by_slot.at(E.slot);
      if (!mk[j]) { mk[j] = 1; work.push_back(j); }
    }
  }
  std::vector<int> par;
  for (int i = 0; i < n; ++i)
    if (mk[i]) par.push_back(i);
  return par;
}
}  // namespace

extern "C" {

mrb_status mrb_refine_marked(mrb_ctx* c, const int8_t* mask, int* n_refined) {
  if (!c || !mask) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (!check_state(c, true)) return MRB_E_STATE;
  std::vector<int> par = graded_closure(c, mask);
  if (n_refined) *n_refined = (int)par.size();
  return do_refine(c, par, true, true, mask);
}

mrb_status mrb_step_predicted(mrb_ctx* c, double t, double dt, float tau, float guard, int* n_refined) {
  if (!c) return MRB_E_ARG;
  if (c->dev.active) {
    mrb_status ps = dev_pull(c);
    if (ps) return ps;
  }
  if (!check_state(c, true)) return MRB_E_STATE;
  if (mlp_ready(c)) return MRB_E_STATE;
  if (!(dt > 0.0)) return fail(c, MRB_E_ARG, "step_predicted: dt must be positive");
  const int n = (int)c->hblk.size();
  std::vector<int8_t> pred(n), mask(n);
  std::vector<float> prob(n);
  mrb_status r = mrb_mlp_predict(c, pred.data(), prob.data());
  if (r) return r;
  // refine what the predictor calls 'refine', everything it is unsure about, and (the
  // exact fallback) every block whose last detail maximum reaches guard x threshold
  // for some field, or all blocks if no analysis of the current grid is at hand
  const int nf = c->cfg.nfields;
  const bool have = c->have_flags && c->last_maxd.size() == (size_t)n * nf;
  for (int i = 0; i < n; ++i) {
    bool m = pred[i] == 0 || prob[i] < tau;
    if (!m && guard > 0.0f) {
      if (!have) m = true;
      else
        for (int f = 0; f < nf; ++f)
          if (!(c->last_maxd[(size_t)i * nf + f] < (double)guard * c->thr[f])) m = true;
    }
    mask[i] = m ? 1 : 0;
  }
  if ((r = mrb_refine_marked(c, mask.data(), n_refined))) return r;
  if ((r = do_rk4(c, t, dt))) return r;
  if ((r = do_adapt(c, nullptr))) return r;
  c->n_steps++;
  return MRB_OK;
}

mrb_status mrb_horizon_labels(int dim, int n_now, const int8_t* lv_now, const int32_t* co_now, int n_later,
                              const int8_t* lv_later, const int32_t* co_later, int8_t* labels) {
  if (dim < 2 || dim > 3 || n_now < 0 || n_later < 0 || !labels) return MRB_E_ARG;
  std::unordered_map<uint64_t, int> later;
  int jmax = 1;
  for (int i = 0; i < n_later; ++i) {
    int c[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) c[a] = co_later[(size_t)i * dim + a];
    later[pack_key(lv_later[i], c)] = lv_later[i];
    jmax = std::max(jmax, (int)lv_later[i]);
  }
  for (int i = 0; i < n_now; ++i) {
    const int l = lv_now[i];
    int c[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) c[a] = co_now[(size_t)i * dim + a];
    bool coarser = false, finer = false;
    for (int L = 1; L < l && !coarser; ++L) {
      int p[3] = {0, 0, 0};
      for (int a = 0; a < dim; ++a) p[a] = c[a] >> (l - L);
      coarser = later.count(pack_key(L, p)) > 0;
    }
    for (int L = l + 1; L <= jmax && !finer; ++L) {
      const int s = L - l, side = 1 << s;
      const long cnt = dim == 2 ? (long)side * side : (long)side * side * side;
      for (long q = 0; q < cnt && !finer; ++q) {
        int cc[3] = {0, 0, 0};
        cc[0] = (c[0] << s) + (int)(q % side);
        cc[1] = (c[1] << s) + (int)((q / side) % side);
        if (dim > 2) cc[2] = (c[2] << s) + (int)(q / ((long)side * side));
        finer = later.count(pack_key(L, cc)) > 0;
      }
    }
    labels[i] = finer ? 0 : (coarser ? 2 : 1);
  }
  return MRB_OK;
}

mrb_status mrb_set_graph(mrb_ctx* c, int enable) {
  if (!c) return MRB_E_ARG;
  if (enable < 0 || enable > 2) return fail(c, MRB_E_ARG, "set_graph: 0 off, 1 on, 2 automatic");
  c->graph_mode = enable;
  c->probe_us[0].clear();
  c->probe_us[1].clear();
  c->use_graph = enable != 0;
  return MRB_OK;
}

mrb_status mrb_set_sweep(mrb_ctx* c, int mode) {
  if (!c) return MRB_E_ARG;
  if (mode < 0 || mode > 3) return fail(c, MRB_E_ARG, "set_sweep: mode must be 0, 1, 2 or 3");
  c->sweep_mode = mode;
  return MRB_OK;
}

mrb_status mrb_set_topology(mrb_ctx* c, int mode) {
  if (!c) return MRB_E_ARG;
  if (mode < 0 || mode > 2) return fail(c, MRB_E_ARG, "set_topology: mode must be 0, 1 or 2");
  c->dev.mode = mode;
  return MRB_OK;
}

mrb_status mrb_timing(mrb_ctx* c, int enable) {
  if (!c) return MRB_E_ARG;
  resolve_timing(c);
  c->timing = enable != 0;
  for (int k = 0; k < T_NKIND; ++k) {
    c->t_ms[k] = 0.0;
    c->t_bytes[k] = 0.0;
    c->t_launches[k] = 0;
  }
  return MRB_OK;
}

}  // extern "C"
