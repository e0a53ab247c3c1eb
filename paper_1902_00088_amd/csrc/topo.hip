// Device-resident topology transitions of the multiresolution step (gfx950): the
// safety-zone refinement plan (Sec. 2.1 item 1), the coarsening plan with its
// completeness and gradedness fixed point (Sec. 2.3, last paragraph; Sec. 2.2 graded
// grid) and the neighbour entries of the new grid, so that a step needs no host
// planning.  The results are the host planner's: the same forest order (Morton), the
// same slots from the same free stack, the same entries in the same order.
//
// Layout: every grid lives in an arena of fixed capacity (header, block descriptors,
// entry rows of a fixed stride, refinement parents with their entry rows, refinement
// and coarsening plans); a dense index holds, for every possible block of every level,
// its position in the current grid or -1; the free pool slots form a stack.
#include "internal.hpp"

#include <hip/hip_runtime.h>

namespace mrb {

namespace {

__device__ __forceinline__ int cell_of(const DevTopoArgs& A, int l, const int* c) {
  int k = A.cell_off[l] + c[0] + (c[1] << l);
  if (A.dim > 2) k += c[2] << (2 * l);
  return k;
}

__device__ __forceinline__ int wrapl(int a, int l) { return a & ((1 << l) - 1); }

// exclusive scan of one value per thread over the workgroup (blockDim.x <= 1024);
// *total receives the sum.  sh: 1024 ints of LDS.
__device__ int wg_scan(int v, int* sh, int* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const int x = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  const int incl = sh[t];
  *total = sh[blockDim.x - 1];
  __syncthreads();
  return incl - v;
}

}  // namespace

// ---------------------------------------------------------------------------
// refinement plan (one workgroup): every block below jmax becomes its 2^dim children
// in its place of the forest order; children take slots from the top of the free
// stack (child ch of the r-th parent takes free[top-1-(r*nch+ch)]), then the parents'
// slots are pushed in forest order.  Writes the new grid's block descriptors (entries
// come later), the refinement plan (children's slots, the parents' descriptors) and
// the new grid's level histogram.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_plan_refine(DevTopoArgs A) {
  __shared__ int sh[1024];
  __shared__ int hist[kMaxLevels];
  const int n = A.old_h.n_blocks, nch = A.nch, t = threadIdx.x, T = blockDim.x;
  const BlockDesc* ob = (const BlockDesc*)(A.old_base + A.old_h.off_blk);
  BlockDesc* nb = (BlockDesc*)(A.new_base + A.new_h.off_blk);
  BlockDesc* pb = (BlockDesc*)(A.new_base + A.new_h.off_pblk);
  RefineDesc* rd = (RefineDesc*)(A.new_base + A.new_h.off_ref);
  int* pmap = A.scratch;   // parent r -> old block index (for the entry-row copy)
  if (t < kMaxLevels) hist[t] = 0;
  // contiguous chunk of blocks per thread: new positions and parent ranks by scans
  const int chunk = (n + T - 1) / T, b0 = min(n, t * chunk), b1 = min(n, b0 + chunk);
  int npos = 0, npar = 0;
  for (int b = b0; b < b1; ++b) {
    const int p = ob[b].level < A.jmax;
    npos += p ? nch : 1;
    npar += p;
  }
  int tot_pos, tot_par;
  int pos = wg_scan(npos, sh, &tot_pos);
  int ri = wg_scan(npar, sh, &tot_par);
  const int top = A.free_top, nref = tot_par;
  for (int b = b0; b < b1; ++b) {
    const BlockDesc d = ob[b];
    if (d.level < A.jmax) {
      RefineDesc r;
      for (int ch = 0; ch < 8; ++ch) r.child[ch] = -1;
      for (int ch = 0; ch < nch; ++ch) {
        BlockDesc k;
        k.slot = A.free_stack[top - 1 - (ri * nch + ch)];
        k.level = d.level + 1;
        k.c[0] = k.c[1] = k.c[2] = 0;
        for (int a = 0; a < A.dim; ++a) k.c[a] = 2 * d.c[a] + ((ch >> a) & 1);
        k.nb_begin = 0;
        k.n_ent = 0;
        k.n_coarse = 0;
        nb[pos + ch] = k;
        r.child[ch] = k.slot;
        atomicAdd(&hist[k.level], 1);
      }
      rd[ri] = r;
      pb[ri] = d;
      pmap[ri] = b;
      ++ri;
      pos += nch;
    } else {
      BlockDesc k = d;
      k.nb_begin = 0;
      k.n_ent = 0;
      k.n_coarse = 0;
      nb[pos] = k;
      atomicAdd(&hist[k.level], 1);
      ++pos;
    }
  }
  __syncthreads();   // every pop above read the stack before the pushes below overwrite it
  {
    int r = wg_scan(npar, sh, &tot_par);
    for (int b = b0; b < b1; ++b) {
      if (ob[b].level >= A.jmax) continue;
      A.free_stack[top - nref * nch + r] = ob[b].slot;
      ++r;
    }
  }
  __syncthreads();
  if (t == 0) {
    A.out[0] = nref;
    A.out[1] = tot_pos;
    A.out[2] = top - nref * nch + nref;
  }
  if (t < kMaxLevels) A.out[4 + t] = hist[t];
}

// ---------------------------------------------------------------------------
// coarsening plan, in four launches.  Complete families whose 2^dim members
// (consecutive in forest order) are all flagged -1 are the candidates.  A candidate
// must go while a finer leaf touching one of its members is not in a live candidate
// (the greatest such set: a demotion only removes a family that no valid subset can
// hold, so the order of demotions does not matter).  Every live family's mother takes
// its first child's place in the forest order; mother k (in forest order, of m) takes
// free[top-m+k], and the children's slots are then pushed in reverse forest order.
// Scratch: fam_of[n], first[n], dead[n], edge count, edges (family, family it needs).
// ---------------------------------------------------------------------------
namespace {
__device__ __forceinline__ bool family_first(const DevTopoArgs& A, const BlockDesc* ob, int n, int b) {
  const BlockDesc d = ob[b];
  if (d.level < 2 || A.flags[b] != -1) return false;
  for (int a = 0; a < A.dim; ++a)
    if (d.c[a] & 1) return false;
  if (b + A.nch > n) return false;
  for (int ch = 1; ch < A.nch; ++ch) {
    const BlockDesc e = ob[b + ch];
    if (e.level != d.level || A.flags[b + ch] != -1) return false;
    for (int a = 0; a < A.dim; ++a)
      if (e.c[a] != d.c[a] + ((ch >> a) & 1)) return false;
  }
  return true;
}
}  // namespace

// 0 (whole grid): whether block b is the first member of a candidate family (kept in
// the edge buffer until the edges overwrite it) and whether its detail norms are finite
__global__ void __launch_bounds__(256) k_coarsen_candidates(DevTopoArgs A) {
  const int n = A.old_h.n_blocks;
  const BlockDesc* ob = (const BlockDesc*)(A.old_base + A.old_h.off_blk);
  int bad = 0;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < n; b += gridDim.x * blockDim.x) {
    A.edges[2 + b] = family_first(A, ob, n, b) ? 1 : 0;
    for (int f = 0; f < A.nf; ++f)
      if (!isfinite(A.maxd[(size_t)b * A.nf + f])) bad = 1;
  }
  if (bad) atomicOr(A.err, 2);   // a non-finite detail norm
}

// 1 (one workgroup): candidates numbered in forest order
__global__ void __launch_bounds__(1024) k_coarsen_families(DevTopoArgs A) {
  __shared__ int sh[1024];
  const int n = A.old_h.n_blocks, nch = A.nch, t = threadIdx.x, T = blockDim.x;
  int* fam_of = A.scratch;
  int* first = A.scratch + n;
  int* dead = A.scratch + 2 * n;
  const int* cand = A.edges + 2;
  const int chunk = (n + T - 1) / T, b0 = min(n, t * chunk), b1 = min(n, b0 + chunk);
  int ncand = 0;
  for (int b = b0; b < b1; ++b) {
    fam_of[b] = -1;
    ncand += cand[b];
  }
  int nfam;
  int f = wg_scan(ncand, sh, &nfam);
  __syncthreads();
  for (int b = b0; b < b1; ++b)
    if (cand[b]) {
      for (int ch = 0; ch < nch; ++ch) fam_of[b + ch] = f;
      first[f] = b;
      dead[f] = 0;
      ++f;
    }
  __syncthreads();
  if (t == 0) {
    A.edges[0] = 0;       // edge count
    A.edges[1] = nfam;    // family count
  }
}

// 2 (whole grid): one work item per (member, entry slot): a finer leaf outside every
// candidate kills the member's family; one inside a candidate becomes an edge
__global__ void __launch_bounds__(256) k_coarsen_edges(DevTopoArgs A) {
  const int n = A.old_h.n_blocks, S = A.old_h.nb_stride;
  const BlockDesc* ob = (const BlockDesc*)(A.old_base + A.old_h.off_blk);
  const int* fam_of = A.scratch;
  int* dead = A.scratch + 2 * n;
  const long total = (long)n * S;
  for (long w = blockIdx.x * (long)blockDim.x + threadIdx.x; w < total; w += (long)gridDim.x * blockDim.x) {
    const int m = (int)(w / S), e = (int)(w % S);
    const int f = fam_of[m];
    if (f < 0) continue;
    const BlockDesc M = ob[m];
    if (e >= M.n_ent) continue;
    const NbEntry E = ((const NbEntry*)(A.old_base + A.old_h.off_nb))[(size_t)m * S + e];
    if (E.dl <= 0) continue;
    int fc[3] = {0, 0, 0};
    for (int a = 0; a < A.dim; ++a) fc[a] = wrapl(2 * M.c[a] + (E.o[a] * 2) / (A.bs - 1), M.level + 1);
    const int j = A.cells[cell_of(A, M.level + 1, fc)];
    const int g = j >= 0 ? fam_of[j] : -1;
    if (g < 0) {
      dead[f] = 1;
    } else if (g != f) {
      const int k = atomicAdd(&A.edges[0], 1);
      A.edges[2 + 2 * k] = f;
      A.edges[3 + 2 * k] = g;
    }
  }
}

// 3 (one workgroup): the fixed point over the edges, then the new forest and the plan
__global__ void __launch_bounds__(1024) k_plan_coarsen(DevTopoArgs A) {
  __shared__ int sh[1024];
  __shared__ int hist[kMaxLevels];
  __shared__ int changed;
  __shared__ unsigned char alive_lds[kAliveLds];
  const int n = A.old_h.n_blocks, nch = A.nch, t = threadIdx.x, T = blockDim.x;
  const BlockDesc* ob = (const BlockDesc*)(A.old_base + A.old_h.off_blk);
  BlockDesc* nb = (BlockDesc*)(A.new_base + A.new_h.off_blk);
  FamilyDesc* fd = (FamilyDesc*)(A.new_base + A.new_h.off_fam);
  const int* fam_of = A.scratch;
  const int* first = A.scratch + n;
  int* dead = A.scratch + 2 * n;
  const int nedge = A.edges[0], nfam = A.edges[1];
  // alive flags in LDS when they fit, else in the dead array (dead == 0 means alive)
  const bool lds = nfam <= kAliveLds;
  if (t < kMaxLevels) hist[t] = 0;
  if (lds)
    for (int q = t; q < nfam; q += T) alive_lds[q] = dead[q] ? 0 : 1;
  __syncthreads();
  auto alive = [&](int q) -> bool { return lds ? alive_lds[q] != 0 : dead[q] == 0; };
  auto kill = [&](int q) {
    if (lds) alive_lds[q] = 0;
    else dead[q] = 1;
  };
  for (;;) {
    if (t == 0) changed = 0;
    __syncthreads();
    for (int k = t; k < nedge; k += T) {
      const int f = A.edges[2 + 2 * k], g = A.edges[3 + 2 * k];
      if (alive(f) && !alive(g)) {
        kill(f);
        changed = 1;
      }
    }
    __syncthreads();
    if (!changed) break;
    __syncthreads();
  }
  const int chunk = (n + T - 1) / T, b0 = min(n, t * chunk), b1 = min(n, b0 + chunk);
  int nemit = 0, nlive = 0;
  for (int b = b0; b < b1; ++b) {
    const int fb = fam_of[b];
    const bool gone = fb >= 0 && alive(fb);
    nemit += gone ? (first[fb] == b ? 1 : 0) : 1;
    nlive += gone && first[fb] == b ? 1 : 0;
  }
  int tot_new, m;
  int pos = wg_scan(nemit, sh, &tot_new);
  int k = wg_scan(nlive, sh, &m);
  const int top = A.free_top;
  if (m > top) {
    // the mothers need more free slots than the pool has: nothing is written
    if (t == 0) {
      A.out[0] = 0;
      A.out[1] = n;
      A.out[2] = top;
      A.out[3] = atomicExch(A.err, 0) | 4;
    }
    return;
  }
  for (int b = b0; b < b1; ++b) {
    const int fb = fam_of[b];
    const bool gone = fb >= 0 && alive(fb);
    if (gone && first[fb] != b) continue;
    BlockDesc d = ob[b];
    if (gone) {
      FamilyDesc F;
      F.parent = A.free_stack[top - m + k];
      for (int ch = 0; ch < 8; ++ch) F.child[ch] = ch < nch ? ob[b + ch].slot : -1;
      fd[k] = F;
      d.slot = F.parent;
      d.level -= 1;
      for (int a = 0; a < A.dim; ++a) d.c[a] >>= 1;
      ++k;
    }
    d.nb_begin = 0;
    d.n_ent = 0;
    d.n_coarse = 0;
    nb[pos++] = d;
    atomicAdd(&hist[d.level], 1);
  }
  __syncthreads();   // the mothers' pops above precede the pushes below
  {
    // children of live family kk go to free[top - m + (m*nch - 1 - (kk*nch + ch))]
    int kk = wg_scan(nlive, sh, &m);
    for (int b = b0; b < b1; ++b) {
      const int fb = fam_of[b];
      if (!(fb >= 0 && alive(fb) && first[fb] == b)) continue;
      for (int ch = 0; ch < nch; ++ch)
        A.free_stack[top - m + (m * nch - 1 - (kk * nch + ch))] = ob[b + ch].slot;
      ++kk;
    }
  }
  __syncthreads();
  if (t == 0) {
    A.out[0] = m;
    A.out[1] = tot_new;
    A.out[2] = top - m + m * nch;
    // errors of this plan and of the entry builds since the last one, reported and cleared
    A.out[3] = atomicExch(A.err, 0);
  }
  if (t < kMaxLevels) A.out[4 + t] = hist[t];
}

// clear (val = -1, grid `old`) or set (val = position, grid `new`) the dense index
__global__ void __launch_bounds__(256) k_index(DevTopoArgs A, int set) {
  const char* base = set ? A.new_base : A.old_base;
  const TopoHeader& h = set ? A.new_h : A.old_h;
  const BlockDesc* bd = (const BlockDesc*)(base + h.off_blk);
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < h.n_blocks; b += gridDim.x * blockDim.x) {
    const BlockDesc d = bd[b];
    A.cells[cell_of(A, d.level, d.c)] = set ? b : -1;
  }
}

// ---------------------------------------------------------------------------
// neighbour entries of the new grid, one wave per block: lane q takes direction q of
// the 3^dim block neighbourhood (x fastest) -- a same-level leaf, else the coarser
// leaf covering that position (once per distinct leaf and image), else the finer
// leaves touching the block there -- and the wave writes them in the order the
// kernels rely on: coarser, the block itself, same level, finer, each in direction
// order.  Waves past the blocks copy the refinement parents' entry rows.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_entries(DevTopoArgs A) {
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  const int nblk = A.new_h.n_blocks, nref = A.new_h.n_ref;
  const int S = A.new_h.nb_stride;
  const int nd = A.dim == 2 ? 9 : 27, center = nd / 2;
  const BlockDesc* bd = (const BlockDesc*)(A.new_base + A.new_h.off_blk);
  for (int w = blockIdx.x * wpb + (threadIdx.x >> 6); w < nblk + nref; w += gridDim.x * wpb) {
    if (w >= nblk) {
      // refinement parent r: its entry row on the grid before refinement
      const int r = w - nblk;
      const int b = A.scratch[r];
      const NbEntry* src = (const NbEntry*)(A.old_base + A.old_h.off_nb) + (size_t)b * A.old_h.nb_stride;
      NbEntry* dst = (NbEntry*)(A.new_base + A.new_h.off_pnb) + (size_t)r * A.new_h.pnb_stride;
      for (int e = lane; e < A.old_h.nb_stride; e += 64) dst[e] = src[e];
      continue;
    }
    const BlockDesc L = bd[w];
    const int l = L.level, bs1 = A.bs - 1;
    int dlt[3] = {0, 0, 0};
    bool act = lane < nd && lane != center;
    if (lane < nd) {
      dlt[0] = lane % 3 - 1;
      dlt[1] = (lane / 3) % 3 - 1;
      dlt[2] = A.dim > 2 ? lane / 9 - 1 : 0;
    }
    int cn[3] = {0, 0, 0};
    for (int a = 0; a < A.dim; ++a) cn[a] = L.c[a] + dlt[a];
    // same level
    int sslot = -1, cslot = -1, nfine = 0, err = 0;
    NbEntry fine[4];
    int8_t co[3] = {0, 0, 0};
    if (act) {
      int wc[3] = {0, 0, 0};
      for (int a = 0; a < A.dim; ++a) wc[a] = wrapl(cn[a], l);
      const int j = A.cells[cell_of(A, l, wc)];
      if (j >= 0) {
        sslot = bd[j].slot;
      } else {
        bool found = false;
        if (l > 1) {
          int pc[3] = {0, 0, 0}, wp[3] = {0, 0, 0};
          for (int a = 0; a < A.dim; ++a) {
            pc[a] = cn[a] >> 1;   // floor division
            wp[a] = wrapl(pc[a], l - 1);
          }
          const int jc = A.cells[cell_of(A, l - 1, wp)];
          if (jc >= 0) {
            cslot = bd[jc].slot;
            for (int a = 0; a < A.dim; ++a) co[a] = (int8_t)((2 * pc[a] - L.c[a]) * bs1);
            found = true;
          }
        }
        if (!found) {
          if (l >= A.jmax) err = 1;
          for (int b = 0; b < (1 << A.dim) && !err; ++b) {
            int beta[3] = {0, 0, 0};
            bool ok = true;
            for (int a = 0; a < A.dim; ++a) {
              beta[a] = (b >> a) & 1;
              if (dlt[a] == 1 && beta[a] != 0) ok = false;
              if (dlt[a] == -1 && beta[a] != 1) ok = false;
            }
            if (!ok) continue;
            int ch[3] = {0, 0, 0};
            for (int a = 0; a < A.dim; ++a) ch[a] = 2 * wrapl(cn[a], l) + beta[a];
            const int jf = A.cells[cell_of(A, l + 1, ch)];
            if (jf < 0) {
              err = 1;
              break;
            }
            NbEntry e;
            e.slot = bd[jf].slot;
            e.dl = 1;
            e.o[0] = e.o[1] = e.o[2] = 0;
            for (int a = 0; a < A.dim; ++a) e.o[a] = (int8_t)(dlt[a] * bs1 + beta[a] * (bs1 / 2));
            if (nfine < 4) fine[nfine] = e;
            ++nfine;
          }
        }
      }
    }
    // a coarser leaf reached from several directions (same slot and origin) counts once
    const int ckey = cslot >= 0 ? ((int)(uint8_t)co[0] | ((int)(uint8_t)co[1] << 8) | ((int)(uint8_t)co[2] << 16)) : 0;
    bool keep_c = cslot >= 0;
    for (int q = 0; q < nd; ++q) {
      const int os = __shfl(cslot, q, 64), ok = __shfl(ckey, q, 64);
      if (q < lane && keep_c && os == cslot && ok == ckey) keep_c = false;
    }
    // positions: exclusive prefix sums over the lanes
    const unsigned long long below = (1ull << lane) - 1ull;
    const unsigned long long bc = __ballot(keep_c), bsm = __ballot(sslot >= 0);
    const int nc_before = __popcll(bc & below), ncoarse = __popcll(bc);
    const int ns_before = __popcll(bsm & below), nsame = __popcll(bsm);
    int fpre = nfine;
    for (int off = 1; off < 64; off <<= 1) {
      const int x = __shfl_up(fpre, off, 64);
      if (lane >= off) fpre += x;
    }
    const int nfine_all = __shfl(fpre, 63, 64);
    fpre -= nfine;
    const int errs = __popcll(__ballot(err != 0));
    NbEntry* row = (NbEntry*)(A.new_base + A.new_h.off_nb) + (size_t)w * S;
    const int nent = ncoarse + 1 + nsame + nfine_all;
    if (errs || nent > S) {
      if (lane == 0) atomicOr(A.err, 1);   // not graded, or a hole
      continue;
    }
    if (keep_c) {
      NbEntry e;
      e.slot = cslot;
      e.dl = -1;
      e.o[0] = co[0];
      e.o[1] = co[1];
      e.o[2] = co[2];
      row[nc_before] = e;
    }
    if (lane == 0) {
      NbEntry e;
      e.slot = L.slot;
      e.dl = 0;
      e.o[0] = e.o[1] = e.o[2] = 0;
      row[ncoarse] = e;
    }
    if (sslot >= 0) {
      NbEntry e;
      e.slot = sslot;
      e.dl = 0;
      e.o[0] = e.o[1] = e.o[2] = 0;
      for (int a = 0; a < A.dim; ++a) e.o[a] = (int8_t)(dlt[a] * bs1);
      row[ncoarse + 1 + ns_before] = e;
    }
    for (int i = 0; i < nfine && i < 4; ++i) row[ncoarse + 1 + nsame + fpre + i] = fine[i];
    if (lane == 0) {
      BlockDesc d = L;
      d.nb_begin = w * S;
      d.n_ent = nent;
      d.n_coarse = ncoarse;
      ((BlockDesc*)(A.new_base + A.new_h.off_blk))[w] = d;
    }
  }
}

// fill n ints with a value
__global__ void __launch_bounds__(256) k_fill_int(int* p, size_t n, int v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_plan_refine(const DevTopoArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_plan_refine, dim3(1), dim3(1024), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_plan_coarsen(const DevTopoArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_coarsen_candidates, dim3(grid > 0 ? grid : 1), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_coarsen_families, dim3(1), dim3(1024), 0, st, a);
  hipLaunchKernelGGL(k_coarsen_edges, dim3(grid > 0 ? grid : 1), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_plan_coarsen, dim3(1), dim3(1024), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_index(const DevTopoArgs& a, int set, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_index, dim3(grid > 0 ? grid : 1), dim3(256), 0, st, a, set);
  return hipGetLastError();
}

hipError_t launch_entries(const DevTopoArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_entries, dim3(grid > 0 ? grid : 1), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, size_t n, int v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int grid = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_fill_int, dim3(grid), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace mrb
