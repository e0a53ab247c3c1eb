// Internal types shared by the host forest manager (mrb.cpp) and the HIP kernels
// (kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mrb {

constexpr int kMaxLevels = 16;
constexpr int kMaxEnt = 64;   // neighbour entries per block (3D needs at most 57)

// One active block, in forest (Morton) order.
struct BlockDesc {
  int slot;       // pool slot of the block's data
  int level;
  int c[3];       // integer coordinates at its level
  int nb_begin;   // first neighbour entry in the host's packed list
  int n_ent;      // entries: coarser leaves first, then same-level leaves (the block
  int n_coarse;   // itself included), then finer leaves
};

// A leaf whose closed region touches the block (diagonal neighbours included).
// Its region is [o, o + ext]^dim in the block's level-l node units, with
// ext = (bs-1) * 2^-dl.  Periodic images are separate entries.
struct NbEntry {
  int slot;
  int8_t dl;      // level(neighbour) - level(block): -1, 0 or +1
  int8_t o[3];    // |o| <= 2 (bs-1) <= 124 (bs <= 63)
};
static_assert(sizeof(NbEntry) == 8, "NbEntry packs into 8 bytes");

// Refinement work r: the slots of the 2^dim children of parent r of the parent
// section (child bit a = coordinate bit along axis a).
struct RefineDesc {
  int child[8];
};

// Coarsening of one family: the new mother's slot and the children's slots.
struct FamilyDesc {
  int parent;
  int child[8];
};

// Header of the packed topology buffer (one host->device copy per topology change).
// Offsets are in bytes from the start of the buffer.  Block b's neighbour entries sit
// at off_nb + b * nb_stride entries (nb_stride = the largest entry count of the
// upload), and refinement r's parent entries at off_pnb + r * pnb_stride, so a
// kernel can load a block's descriptor and its entries at the same time.
struct TopoHeader {
  int n_blocks;   // current grid
  int n_ref;      // refinement work items
  int n_fam;      // coarsening families
  int n_pblk;     // parents (refinement); parent r belongs to refinement r
  int off_blk, off_nb, off_list, off_pblk, off_pnb, off_ref, off_fam;
  int nb_stride, pnb_stride;
  int off_smap;   // coarsening uploads: per block of the grid before, mother slot * 8 +
                  // child index or -1 (read by a later analysis that speculates it); 0: none
  int pad[2];
};
static_assert(sizeof(TopoHeader) == 64, "the header is 64 bytes (graph keys hold it as 8 words)");

// Kernel view of the topology: the buffer and a copy of its header, passed by value
// so that no launch waits on a load of the header.
struct Topo {
  const char* base;
  TopoHeader h;
  __device__ __forceinline__ const BlockDesc* blk() const { return (const BlockDesc*)(base + h.off_blk); }
  __device__ __forceinline__ const NbEntry* nb(int b) const {
    return (const NbEntry*)(base + h.off_nb) + (size_t)b * h.nb_stride;
  }
  __device__ __forceinline__ const int* list() const { return (const int*)(base + h.off_list); }
  __device__ __forceinline__ const BlockDesc* pblk() const { return (const BlockDesc*)(base + h.off_pblk); }
  __device__ __forceinline__ const NbEntry* pnb(int r) const {
    return (const NbEntry*)(base + h.off_pnb) + (size_t)r * h.pnb_stride;
  }
  __device__ __forceinline__ const RefineDesc* ref() const { return (const RefineDesc*)(base + h.off_ref); }
  __device__ __forceinline__ const FamilyDesc* fam() const { return (const FamilyDesc*)(base + h.off_fam); }
};

struct LevelTab {
  double r[kMaxLevels];   // 1/(12 h_l) = N_l / 12
  float rf[kMaxLevels];
  int nl[kMaxLevels];     // N_l = 2^l (bs-1)
};

struct Physics {
  int kind;               // MRB_ADV_CONST / MRB_ADV_SWIRL / MRB_NS2D
  double c[3];            // advection velocity
  const double* s2;       // device swirl tables (finest lattice)
  const double* s;
  int jmax;
  double gamma, mu, kap;  // NS: gamma, viscosity, mu*gamma/((gamma-1) Pr)
};

// Arguments of one RK stage sweep.  Stage s builds y = u + alpha * kprev
// (stage 1: y = u) over block + halo and evaluates the RHS; stages 1-3 store
// k_s into kout, stage 4 stores u + h6*((k1 + k4) + 2 (k2 + k3)) into unew.
struct StageArgs {
  Topo topo;
  int lvl_begin, lvl_end; // plain form: range of the level-sorted block list (else 0, -1)
  int order;              // fused form: 0 forest (Morton) order, 1 level-sorted order
  const double* u;
  const void* kprev;
  double alpha;
  void* kout;
  const void* k1;
  const void* k2;
  const void* k3;
  double* unew;
  double h6;
  int stage;              // 1..4
  double cfac;            // swirl time factor for this stage
  double off[4];          // mixed precision: per-field offsets
  LevelTab lt;
  Physics ph;
  double* ghost;          // plain form: ghosted stage values [slot][f][(bs+2hw)^dim]
};

// Whole-sweep launch: the four stages in one kernel with grid barriers between them.
constexpr int kBarStride = 32;   // barrier words 128 bytes apart: 8 group counts, the top count, the generation
constexpr int kBarWords = 10 * kBarStride;
struct SweepArgs {
  StageArgs a;            // stage-independent fields (k1..k3, u, unew, h6, topology, physics)
  double alpha[4];        // y_s = u + alpha_s k_{s-1}
  double cfac[4];         // swirl time factor per stage
  unsigned* bar;          // [kBarWords] device words, counts zero between launches
  int* err;               // set to 1 when a barrier wait times out
  unsigned spin;          // polls before a barrier wait gives up
};

// One-launch RK4 step over overlapped tiles (2D advection on a forest whose leaves
// are all on one level): u over the region plus 4 halo widths, every stage in LDS.
struct Rk4tArgs {
  Topo topo;
  const double* u;
  double* unew;
  double alpha[4];        // y_s = u + alpha_s k_{s-1}
  double cfac[4];         // swirl time factor per stage
  double h6;
  double off;             // FP32 tile offset (one field)
  LevelTab lt;
  Physics ph;
  // with the analysis of u_new folded in (the first pass of an adapt): flags and
  // maxima as MrArgs where a block is one workgroup's region; with sub-tiles, each
  // sub-tile's maximum |detail| instead, per block and sub-tile (mapped host memory,
  // plain stores), and the host takes the maximum and applies the flag rule
  int8_t* flags;
  double* maxd;
  double* part;
  double thr;
  const int* smap;
  // with the speculated coarsening's second analysis folded in as well (every block
  // merges): per block and sub-tile, the maximum |detail| of the mother's nodes the
  // sub-tile holds (mapped host memory, plain stores)
  double* mq;
};

struct MrArgs {
  Topo topo;
  double* u;              // read; redundant nodes owned by finer blocks are written back
  int8_t* flags;          // [n]
  double* maxd;           // [n][nf]
  unsigned long long* acc;// [max_blocks][nf] partial maxima (bit patterns), zero between passes
  int* done;              // [max_blocks] sub-tiles finished, zero between passes
  double thr[4];
  const int* smap;        // [n] speculated coarsening whose mothers the pass writes:
                          // mother slot * 8 + child index of block b, or -1; null: none
};

struct RefineArgs {
  Topo topo;
  double* u;
};

struct CoarsenArgs {
  Topo topo;
  double* u;
};

// shock-capturing filter of the Navier-Stokes shape: reads u, writes unew
struct FilterArgs {
  Topo topo;
  const double* u;
  double* unew;
  double rth;             // sensor threshold
};

struct ReadArgs {
  Topo topo;
  const double* u;
  double* out;            // level 0: [n][nf][bs^dim]; level L > 0: [nf][N_L^dim], x fastest
  int level;              // 0: per block; L: uniform lattice of level L (no leaf coarser than L)
};

struct Shape {
  int dim, bs, hw, nf;
};

// Kernel variant of the stage sweep: sub-tiles per axis (1, 2 or 4).
struct Variant {
  int nsub;
  int tpb = 256;          // threads per workgroup (stage kernel)
};

// Launchers (kernels.hip).  grid = number of workgroups (grid-stride loops inside).
hipError_t launch_stage(const Shape& s, int precision, Variant v, int grid, const StageArgs& a, hipStream_t st);
// Whole-sweep kernel, cooperative launch of at most one workgroup per compute unit
// (and at most `max_grid`); *grid_out gets the count.  hipErrorInvalidValue if the
// variant is not compiled.
hipError_t launch_sweep(const Shape& s, int precision, Variant v, int max_grid, const SweepArgs& a, hipStream_t st,
                        int* grid_out);
hipError_t launch_plain(const Shape& s, int grid, const StageArgs& a, hipStream_t st);  // ghost + RHS kernels
// overlapped-tile RK4 step; hipErrorInvalidValue if the shape has no such kernel
// (threads per workgroup: 256; with the analysis on whole blocks also 512 or 1024;
// refine: the refinement of the parents (every one, a forest on one level) folded in,
// with the analysis only; mothers: the second analysis of a speculated coarsening that
// merges every block, with refine only)
hipError_t launch_rk4t(const Shape& s, int precision, int nsub, bool analysis, bool refine, bool mothers, int tpb,
                       int grid, const Rk4tArgs& a, hipStream_t st);
int rk4t_variants(const Shape& s, int precision, int* nsub, int cap);
hipError_t launch_mr(const Shape& s, int nsub, int tpb, int grid, const MrArgs& a, hipStream_t st);
int mr_threads(const Shape& s, int nsub, int* tpb, int cap);   // compiled workgroup sizes (256 first)
hipError_t launch_refine(const Shape& s, int nsub, int grid, const RefineArgs& a, hipStream_t st);
hipError_t launch_coarsen(const Shape& s, int grid, const CoarsenArgs& a, hipStream_t st);
hipError_t launch_read(const Shape& s, int grid, const ReadArgs& a, hipStream_t st);
hipError_t launch_filter(const Shape& s, int grid, const FilterArgs& a, hipStream_t st);   // NS shape only
hipError_t launch_scatter(const double* src, const int* slots, int n, size_t bsz, double* dst, hipStream_t st);
// Device-resident topology transitions (topo.hip).  Arenas share the TopoHeader layout;
// old_* is the current grid, new_* the next one.
struct DevTopoArgs {
  const char* old_base;
  TopoHeader old_h;
  char* new_base;
  TopoHeader new_h;
  int* cells;                       // dense index: position in the current grid, or -1
  int cell_off[kMaxLevels + 1];     // first cell of each level
  int* free_stack;
  int free_top;                     // entries in the free stack at launch
  const int8_t* flags;              // analysis flags of the current grid (coarsening plan)
  const double* maxd;               // and its detail maxima [n][nf] (checked for finiteness)
  int nf;
  int* scratch;                     // [3 * max_blocks] ints
  int* edges;                       // [2 + 2 * max_blocks * entry stride] ints (coarsening plan;
                                    // first the candidates, then the edges)
  int* err;                         // device word: error bits (1 not graded, 2 non-finite detail
                                    // norm; the coarsening plan adds 4: too few free slots)
  int* out;                         // mapped host ints (plain stores only): [0] parents or families,
                                    // [1] new block count, [2] new free-stack top, [3] error bits
                                    // (the coarsening plan moves and clears *err), [4..) level histogram
  int dim, bs, jmax, nch;
};
hipError_t launch_plan_refine(const DevTopoArgs& a, hipStream_t st);
hipError_t launch_plan_coarsen(const DevTopoArgs& a, int grid, hipStream_t st);   // four launches
hipError_t launch_index(const DevTopoArgs& a, int set, int grid, hipStream_t st);   // set 0: clear old, 1: set new
hipError_t launch_entries(const DevTopoArgs& a, int grid, hipStream_t st);
hipError_t launch_fill_int(int* p, size_t n, int v, hipStream_t st);
constexpr int kDevOutInts = 4 + kMaxLevels;
constexpr int kAliveLds = 32768;   // families whose live flags the coarsening plan keeps in LDS

// Library-owned device scratch of kScratchBytes per GPU (a static device array, no
// allocation): scratch_setup stores its address on the current device in *out.
constexpr size_t kScratchBytes = (size_t)2 << 20;
hipError_t scratch_setup(void** out);
// zero `bytes` (a multiple of 4) at p with a fill kernel
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
bool shape_supported(const Shape& s);
// sub-tile counts compiled for this shape and precision; returns count
int stage_variants(const Shape& s, int precision, int* nsub, int cap);
// threads-per-workgroup choices compiled for a stage tiling (256 always among them)
int stage_threads(const Shape& s, int precision, int nsub, int* tpb, int cap);
// sub-tile counts of the analysis (kind 0) and refinement (kind 1) kernels
int aux_variants(const Shape& s, int kind, int* nsub, int cap);

}  // namespace mrb
