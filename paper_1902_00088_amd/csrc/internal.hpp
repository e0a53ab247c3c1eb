// Internal types shared by the host forest manager (mrb.cpp) and the HIP kernels
// (kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mrb {

constexpr int kMaxLevels = 16;
constexpr int kNT = 256;  // threads per workgroup of the block kernels (4 wave64)

// One active block of the current grid, in forest (Morton) order.
struct BlockDesc {
  int slot;       // pool slot of the block's data
  int level;
  int c[3];       // integer coordinates at its level
  int nb_begin;   // first neighbour entry
  int n_coarse;   // entries are stored coarser leaves first,
  int n_same;     // then same-level leaves (the block itself included),
  int n_fine;     // then finer leaves
};

// A leaf whose closed region touches the block (diagonal neighbours included).
// Its region is [o, o + ext]^dim in the block's level-l node units, with
// ext = (bs-1) * 2^-dl.  Periodic images are separate entries.
struct NbEntry {
  int slot;
  int dl;         // level(neighbour) - level(block): -1, 0 or +1
  int o[3];
};

// Refinement of one block of the previous grid: its descriptor index and the
// slots of its 2^dim children (child bit a = coordinate bit along axis a).
struct RefineDesc {
  int blk;
  int child[8];
};

// Coarsening of one family: the new mother's slot and the children's slots.
struct FamilyDesc {
  int parent;
  int child[8];
};

struct LevelTab {
  double r[kMaxLevels];   // 1/(12 h_l) = N_l / 12
  float rf[kMaxLevels];
  int nl[kMaxLevels];     // N_l = 2^l (bs-1)
};

struct Physics {
  int kind;               // MRB_ADV_CONST / MRB_ADV_SWIRL / MRB_NS2D
  double c[3];            // advection velocity
  float cf[3];
  const double* s2;       // device swirl tables (finest lattice)
  const double* s;
  int jmax;
  double gamma, mu, kap;  // NS: gamma, viscosity, mu*gamma/((gamma-1) Pr)
};

// Arguments of one RK stage sweep.  Stage s builds y = u + alpha * kprev
// (stage 1: y = u) over block + halo and evaluates the RHS; stages 1-3 store
// k_s into kout, stage 4 stores u + h6*((k1 + k4) + 2 (k2 + k3)) into unew.
struct StageArgs {
  const BlockDesc* blk;
  const NbEntry* nb;
  const int* count;       // device: number of blocks
  const int* list;        // optional block-index list (plain form per level), else null
  int list_n;
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

struct MrArgs {
  const BlockDesc* blk;
  const NbEntry* nb;
  const int* count;
  double* u;              // read; redundant nodes owned by finer blocks are written back
  int8_t* flags;          // [n]
  double* maxd;           // [n][nf]
  double thr[4];
};

struct RefineArgs {
  const BlockDesc* blk;   // descriptors of the grid before refinement
  const NbEntry* nb;
  const RefineDesc* ref;
  const int* count;       // device: number of refined blocks
  double* u;
};

struct CoarsenArgs {
  const FamilyDesc* fam;
  const int* count;
  double* u;
};

struct ReadArgs {
  const BlockDesc* blk;
  const NbEntry* nb;
  const int* count;
  const double* u;
  double* out;            // [n][nf][bs^dim]
};

// Kernel variant key: one compiled instantiation per supported shape.
struct Shape {
  int dim, bs, hw, nf;
};

// Launchers (kernels.hip).  Each returns a hipError_t; grid = number of workgroups.
hipError_t launch_stage(const Shape& s, int precision, int form_plain_rhs, int grid, const StageArgs& a,
                        hipStream_t st);
hipError_t launch_ghost(const Shape& s, int grid, const StageArgs& a, hipStream_t st);
hipError_t launch_mr(const Shape& s, int grid, const MrArgs& a, hipStream_t st);
hipError_t launch_refine(const Shape& s, int grid, const RefineArgs& a, hipStream_t st);
hipError_t launch_coarsen(const Shape& s, int grid, const CoarsenArgs& a, hipStream_t st);
hipError_t launch_read(const Shape& s, int grid, const ReadArgs& a, hipStream_t st);
bool shape_supported(const Shape& s);

}  // namespace mrb
