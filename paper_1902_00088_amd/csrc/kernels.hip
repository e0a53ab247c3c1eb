// HIP kernels of the block-multiresolution sweep (gfx950).
//
// A workgroup handles one block (or one sub-tile of a block) per iteration of a
// grid-stride loop, so a launch does not depend on the block count (it is read from
// the device topology header) and can be replayed from a graph.
//
// Ghost synchronisation is a single gather into LDS.  The block's neighbour
// entries (every leaf whose closed region touches the block: coarser leaves first,
// then same-level leaves including the block itself, then finer leaves) are loaded
// into LDS, and for each axis a 64-bit mask per tile coordinate records which
// entries hold that coordinate on their own lattice.  The owner of a tile point is
// the highest set bit of the AND of its axis masks: the finest leaf holding the
// point (finer blocks own the redundant nodes, Sec. 2.2 and Sec. 2.5).  All loads of
// a tile are issued in one round.  A point held by no leaf lies inside a coarser
// leaf off its lattice and is predicted from the gathered coarse-lattice points by
// the 4th-order central midpoint rule, tensor product x -> y -> z (the prediction
// operator of Sec. 2.3).  The stencil work is bandwidth bound and uses plain vector
// ALUs (no MFMA).
#include "internal.hpp"

#include <hip/hip_runtime.h>
#include <algorithm>
#include <mutex>


namespace mrb {

template <int DIM, int N>
struct Pow { static constexpr int v = N * Pow<DIM - 1, N>::v; };
template <int N>
struct Pow<0, N> { static constexpr int v = 1; };

// midpoint prediction from four equidistant points (cubic through a, b, c, d)
__device__ __forceinline__ double P4(double a, double b, double c, double d) {
  return (9.0 * (b + c) - (a + d)) * 0.0625;
}
__device__ __forceinline__ float P4(float a, float b, float c, float d) {
  return (9.0f * (b + c) - (a + d)) * 0.0625f;
}
// 4th-order central first derivative, r = 1/(12 h)
__device__ __forceinline__ double D4(double um2, double um1, double up1, double up2, double r) {
  return (8.0 * (up1 - um1) - (up2 - um2)) * r;
}
__device__ __forceinline__ float D4(float um2, float um1, float up1, float up2, float r) {
  return (8.0f * (up1 - um1) - (up2 - um2)) * r;
}

// Tensor-product prediction: per axis either one point (n = 1) or four points
// base + q*stride (n = 4) combined by P4; x first, then y, then z.  The number of
// points per axis is fixed at compile time (fully unrolled).
template <int NX, int NY, int NZ, typename T, typename AT>
__device__ __forceinline__ T tensor_fixed(const AT& at, const int* base, const int* stride) {
  T vz[4];
#pragma unroll
  for (int iz = 0; iz < NZ; ++iz) {
    T vy[4];
#pragma unroll
    for (int iy = 0; iy < NY; ++iy) {
      T vx[4];
#pragma unroll
      for (int ix = 0; ix < NX; ++ix)
        vx[ix] = at(base[0] + ix * stride[0], base[1] + iy * stride[1], base[2] + iz * stride[2]);
      vy[iy] = NX == 4 ? P4(vx[0], vx[1], vx[2], vx[3]) : vx[0];
    }
    vz[iz] = NY == 4 ? P4(vy[0], vy[1], vy[2], vy[3]) : vy[0];
  }
  return NZ == 4 ? P4(vz[0], vz[1], vz[2], vz[3]) : vz[0];
}

// p / d for 0 <= p < 2^21 and d >= 1, through the float reciprocal rd = fl(1/d):
// (p + 1/2)/d lies at least 1/(2d) from an integer, and the two roundings (of 1/d and
// of the product) move it by at most (p + 1/2)/d * 2^-23, less than that.  Index splits
// by sizes known only at run time use it: an integer division costs tens of
// instructions per point.
__device__ __forceinline__ int fdiv(int p, float rd) { return (int)(((float)p + 0.5f) * rd); }

// Nodes of [r0, r0+cnt) whose parity pattern is `cls` (bit a set: odd along axis a):
// per-axis first coordinate and count, for a loop without divergence between classes.
template <int DIM>
struct ParityClass {
  int first[3], n[3], total;
  float rn0, rn01;
  __device__ __forceinline__ ParityClass(int cls, const int* r0, const int* cnt) {
    total = 1;
    for (int a = 0; a < 3; ++a) { first[a] = 0; n[a] = 1; }
    for (int a = 0; a < DIM; ++a) {
      const int odd = (cls >> a) & 1;
      first[a] = r0[a] + (((r0[a] & 1) != odd) ? 1 : 0);
      const int last = r0[a] + cnt[a] - 1;
      n[a] = first[a] <= last ? (last - first[a]) / 2 + 1 : 0;
      total *= n[a];
    }
    // (an empty class runs no point, its reciprocals are unused)
    rn0 = 1.0f / (float)n[0];
    rn01 = 1.0f / (float)(n[0] * n[1]);
  }
  __device__ __forceinline__ void coords(int p, int* t) const {
    const int q0 = fdiv(p, rn0);  // p / n[0]
    t[0] = first[0] + 2 * (p - q0 * n[0]);
    if (DIM > 2) {
      const int q1 = fdiv(p, rn01);  // p / (n[0] n[1])
      t[1] = first[1] + 2 * (q0 - q1 * n[1]);
      t[2] = first[2] + 2 * q1;
    } else {
      t[1] = first[1] + 2 * q0;
      t[2] = 0;
    }
  }
};

// Run body.template operator()<NX, NY, NZ>(cls) for every parity class except all-even.
template <int DIM, typename B>
__device__ __forceinline__ void for_odd_classes(B& body) {
  body.template go<4, 1, 1>(1);
  body.template go<1, 4, 1>(2);
  body.template go<4, 4, 1>(3);
  if constexpr (DIM > 2) {
    body.template go<1, 1, 4>(4);
    body.template go<4, 1, 4>(5);
    body.template go<1, 4, 4>(6);
    body.template go<4, 4, 4>(7);
  }
}

// maximum that propagates NaN (a NaN detail must block coarsening)
__device__ __forceinline__ double nanmax(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}

// Tile over a region of S nodes per axis (block-local origin r0) with a halo of H.
template <int DIM, int BS, int S, int H>
struct Geo {
  static constexpr int TW = S + 2 * H;
  static constexpr int TSZ = Pow<DIM, TW>::v;
  static constexpr int NP = Pow<DIM, BS>::v;
  __device__ static __forceinline__ int idx(int ix, int iy, int iz) {  // tile coordinates
    return ix + TW * iy + (DIM > 2 ? TW * TW * iz : 0);
  }
};

template <int DIM, int TW>
struct GState {
  NbEntry ent[kMaxEnt];
  unsigned long long m[DIM][TW];
};

// Stage value source: y = u (+ alpha * k), minus a per-field offset in FP32 tiles.
template <typename TT, typename KT, bool HASK>
struct YSrc {
  const double* u;
  const KT* k;
  double alpha;
  const double* off;
  __device__ __forceinline__ TT operator()(size_t i, int f) const {
    double y = u[i];
    if (HASK) y = y + alpha * (double)k[i];
    if constexpr (sizeof(TT) == 4) return (TT)(y - off[f]);
    else return y;
  }
};

// Load the block's entries and build the per-axis candidate masks of the tile.
template <int DIM, int BS, int S, int H>
__device__ void gsetup(GState<DIM, S + 2 * H>& g, const BlockDesc& d, const NbEntry* ent, int stride, const int* r0) {
  constexpr int TW = S + 2 * H;
  // all `stride` entries of the padded row (in bounds; those past n_ent are unused),
  // so the loads need not wait for the descriptor
  for (int i = threadIdx.x; i < stride; i += blockDim.x) g.ent[i] = ent[i];
  const int ne = d.n_ent;
  __syncthreads();
  // one coordinate per wave and step: lane e tests entry e (at most 64 entries), the
  // wave's ballot is the coordinate's mask
  static_assert(kMaxEnt <= 64, "one entry per lane");
  const int lane = threadIdx.x & 63;
  const bool live = lane < ne;
  const NbEntry E = live ? g.ent[lane] : NbEntry{};   // (lanes past the entries read nothing)
  const int ext = E.dl > 0 ? (BS - 1) / 2 : (E.dl == 0 ? BS - 1 : 2 * (BS - 1));
  for (int q = threadIdx.x >> 6; q < DIM * TW; q += blockDim.x >> 6) {
    const int a = q / TW, it = q % TW, t = r0[a] - H + it;
    const int l = t - (a == 0 ? E.o[0] : (a == 1 ? E.o[1] : E.o[DIM - 1]));
    const unsigned long long mm = __ballot(live && l >= 0 && l <= ext && (E.dl >= 0 || (l & 1) == 0));
    if (lane == 0) g.m[a][it] = mm;
  }
  __syncthreads();
}

// Work items of a launch, XCD-aware: workgroups are dealt round-robin to the 8 XCDs
// (each with its own L2), so XCD x takes the contiguous chunk x of the work list
// (neighbouring blocks in forest order share halo lines in one L2) and its
// workgroups stride through it.  The grid is a multiple of 8.
struct XcdWork {
  int w, end, step;
  __device__ __forceinline__ explicit XcdWork(int total) {
    const int x = blockIdx.x & 7, per = gridDim.x >> 3;
    const int chunk = (total + 7) >> 3;
    w = x * chunk + (blockIdx.x >> 3);
    end = min(total, (x + 1) * chunk);
    step = per;
  }
  __device__ __forceinline__ bool ok() const { return w < end; }
  __device__ __forceinline__ void next() { w += step; }
};

template <int DIM, int TW>
__device__ __forceinline__ unsigned long long cand_at(const GState<DIM, TW>& g, const int* i) {
  unsigned long long c = g.m[0][i[0]] & g.m[1][i[1]];
  if (DIM > 2) c &= g.m[2][i[2]];
  return c;
}

// Gather the tile: every point within hw_all of the region (box A), and the even
// (coarse-lattice) points within h_even (box B, inputs of the prediction; only when
// h_even > hw_all).  A point's owner is the highest set bit of its candidate mask;
// points with no owner are left for gpredict.  Loads go out in batches of B per thread.
template <int DIM, int BS, int S, int H, int NF, typename TT, typename SRC>
__device__ void gfill(TT* tile, const GState<DIM, S + 2 * H>& g, const int* r0, const int* cnt, int hw_all, int h_even,
                      const SRC& src) {
  using G = Geo<DIM, BS, S, H>;
  constexpr int TSZ = G::TSZ, NP = G::NP;
  constexpr int B = 8;
  int a0[3] = {0, 0, 0}, an[3] = {1, 1, 1}, b0[3] = {0, 0, 0}, bn[3] = {1, 1, 1};
  int nA = 1, nB = 0;
  for (int a = 0; a < DIM; ++a) {
    a0[a] = r0[a] - hw_all;
    an[a] = cnt[a] + 2 * hw_all;
    nA *= an[a];
  }
  if (h_even > hw_all) {
    nB = 1;
    for (int a = 0; a < DIM; ++a) {
      const int lo = r0[a] - h_even, hi = r0[a] + cnt[a] - 1 + h_even;
      b0[a] = lo + (lo & 1);
      bn[a] = (hi - b0[a]) / 2 + 1;
      nB *= bn[a];
    }
  }
  const int total = nA + nB;
  const float ra0 = 1.0f / (float)an[0], ra01 = 1.0f / (float)(an[0] * an[1]);
  const float rb0 = 1.0f / (float)bn[0], rb01 = 1.0f / (float)(bn[0] * bn[1]);
  for (int base = 0; base < total; base += B * blockDim.x) {
    size_t addr[B];
    int pos[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int p = base + q * blockDim.x + threadIdx.x;
      pos[q] = -1;
      addr[q] = 0;
      if (p >= total) continue;
      int t[3] = {0, 0, 0};
      if (p < nA) {
        const int q0 = fdiv(p, ra0);
        t[0] = a0[0] + p - q0 * an[0];
        if (DIM > 2) {
          const int q1 = fdiv(p, ra01);
          t[1] = a0[1] + q0 - q1 * an[1];
          t[2] = a0[2] + q1;
        } else {
          t[1] = a0[1] + q0;
        }
      } else {
        const int pb = p - nA;
        const int q0 = fdiv(pb, rb0);
        t[0] = b0[0] + 2 * (pb - q0 * bn[0]);
        if (DIM > 2) {
          const int q1 = fdiv(pb, rb01);
          t[1] = b0[1] + 2 * (q0 - q1 * bn[1]);
          t[2] = b0[2] + 2 * q1;
        } else {
          t[1] = b0[1] + 2 * q0;
        }
        bool inA = true;
        for (int a = 0; a < DIM; ++a)
          if (t[a] < a0[a] || t[a] >= a0[a] + an[a]) inA = false;
        if (inA) continue;  // loaded with box A
      }
      int i[3] = {0, 0, 0};
      for (int a = 0; a < DIM; ++a) i[a] = t[a] - r0[a] + H;
      const unsigned long long cand = cand_at<DIM, S + 2 * H>(g, i);
      if (cand == 0) continue;
      const NbEntry& E = g.ent[63 - __clzll((long long)cand)];
      int sidx = 0, mul = 1;
      for (int a = 0; a < DIM; ++a) {
        const int l = t[a] - E.o[a];
        sidx += (E.dl > 0 ? 2 * l : (E.dl == 0 ? l : l >> 1)) * mul;
        mul *= BS;
      }
      addr[q] = (size_t)E.slot * NF * NP + sidx;
      pos[q] = G::idx(i[0], i[1], i[2]);
    }
    TT v[B][NF];
#pragma unroll
    for (int q = 0; q < B; ++q)
      if (pos[q] >= 0) {
#pragma unroll
        for (int f = 0; f < NF; ++f) v[q][f] = src(addr[q] + (size_t)f * NP, f);
      }
#pragma unroll
    for (int q = 0; q < B; ++q)
      if (pos[q] >= 0) {
#pragma unroll
        for (int f = 0; f < NF; ++f) tile[f * TSZ + pos[q]] = v[q][f];
      }
  }
  __syncthreads();
}

// Predict the points within hw_all of the region that no leaf holds on its lattice,
// one parity class at a time (one unrolled stencil shape per wave).
template <int DIM, int BS, int S, int H, int NF, typename TT>
struct GPredictBody {
  using G = Geo<DIM, BS, S, H>;
  TT* tile;
  const GState<DIM, S + 2 * H>& g;
  const int* r0;
  int a0[3], an[3];
  __device__ __forceinline__ GPredictBody(TT* t_, const GState<DIM, S + 2 * H>& g_, const int* r0_, const int* cnt,
                                          int hw_all)
      : tile(t_), g(g_), r0(r0_) {
    for (int a = 0; a < 3; ++a) { a0[a] = 0; an[a] = 1; }
    for (int a = 0; a < DIM; ++a) {
      a0[a] = r0[a] - hw_all;
      an[a] = cnt[a] + 2 * hw_all;
    }
  }
  template <int NX, int NY, int NZ>
  __device__ __forceinline__ void go(int cls) {
    ParityClass<DIM> pc(cls, a0, an);
    for (int p = threadIdx.x; p < pc.total; p += blockDim.x) {
      int t[3];
      pc.coords(p, t);
      int i[3] = {0, 0, 0};
      for (int a = 0; a < DIM; ++a) i[a] = t[a] - r0[a] + H;
      if (cand_at<DIM, S + 2 * H>(g, i) != 0) continue;
      const int bb[3] = {NX == 4 ? i[0] - 3 : i[0], NY == 4 ? i[1] - 3 : i[1],
                         DIM > 2 ? (NZ == 4 ? i[2] - 3 : i[2]) : 0};
      const int stride[3] = {2, 2, 2};
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const TT* T = tile + f * G::TSZ;
        auto at = [&](int x, int y, int z) { return T[G::idx(x, y, z)]; };
        tile[f * G::TSZ + G::idx(i[0], i[1], i[2])] = tensor_fixed<NX, NY, NZ, TT>(at, bb, stride);
      }
    }
  }
};

template <int DIM, int BS, int S, int H, int NF, typename TT>
__device__ void gpredict(TT* tile, const GState<DIM, S + 2 * H>& g, const int* r0, const int* cnt, int hw_all) {
  GPredictBody<DIM, BS, S, H, NF, TT> body(tile, g, r0, cnt, hw_all);
  for_odd_classes<DIM>(body);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Stage-kernel gather.  The tile holds box A only (the region plus the stencil
// halo HW); the coarse-lattice values that predictions need (even points up to
// H = HW + 3 beyond the region) sit in a compact array C of half resolution, so
// the tile of a block without coarser neighbours carries no prediction margin.
// ---------------------------------------------------------------------------
template <int DIM, int BS, int S, int HW>
struct SGeo {
  static constexpr int H = HW + 3;
  static constexpr int TW = S + 2 * HW;           // tile (box A) width
  static constexpr int TSZ = Pow<DIM, TW>::v;
  static constexpr int CW = (S + 2 * H + 1) / 2;  // coarse-lattice array width
  static constexpr int CSZ = Pow<DIM, CW>::v;
  static constexpr int NP = Pow<DIM, BS>::v;
  __device__ static __forceinline__ int idx(int ix, int iy, int iz) {
    return ix + TW * iy + (DIM > 2 ? TW * TW * iz : 0);
  }
  __device__ static __forceinline__ int cidx(int ix, int iy, int iz) {
    return ix + CW * iy + (DIM > 2 ? CW * CW * iz : 0);
  }
};

// Source address of a held point as base + sum_a f(t_a) BS^a, with f(t) = 2t for a
// finer holder, t for a same-level one and t/2 (floor) for a coarser one (its points are
// even); f(t) = (2t) >> sh with sh = 1 - dl.  The holder's origin is folded into base.
struct SEnt {
  int base;
  int sh;   // 2 coarser, 1 same level, 0 finer
};

template <int DIM, int BS, int NF>
__device__ __forceinline__ void sent_setup(SEnt* se, const NbEntry* ent, int ne) {
  constexpr int NP = Pow<DIM, BS>::v;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    const NbEntry E = ent[e];
    const int sh = 1 - E.dl;
    int b = E.slot * NF * NP, mul = 1;
    for (int a = 0; a < DIM; ++a) {
      b -= ((2 * E.o[a]) >> sh) * mul;
      mul *= BS;
    }
    se[e] = SEnt{b, sh};
  }
}

// Fill box A (and, for blocks with coarser neighbours, the coarse-lattice array).
// Points strictly inside the block are the block's own; the others take their
// owner's value (highest set bit of the candidate mask).  Unowned points of box A
// are left for spredict.  Box A goes row by row: a lane keeps one x position (its
// mask word and x-dependent terms stay in registers) and walks rows of its row
// group; B rows per round, loads issued unconditionally (a lane with no point
// loads the block's first node and discards it).
template <int DIM, int BS, int S, int HW, int NF, bool HASC, typename TT, int B = 8, int NT = 256, typename SRC>
__device__ void sgather(TT* tile, TT* carr, const GState<DIM, S + 2 * (HW + 3)>& g, const SEnt* se, int slot,
                        const int* r0, const int* cnt, const SRC& src) {
  using G = SGeo<DIM, BS, S, HW>;
  constexpr int TW = G::TW, TSZ = G::TSZ, CW = G::CW, CSZ = G::CSZ, NP = G::NP, H = G::H;
  constexpr int RG = NT / TW, NROW = Pow<DIM - 1, TW>::v;
  static_assert(RG >= 1, "tile row wider than the workgroup");
  const int self = slot * NF * NP;
  int cb0[3] = {0, 0, 0};
  for (int a = 0; a < DIM; ++a) cb0[a] = (r0[a] - H + 1) & ~1;
  const int tid = threadIdx.x;
  const int x = tid % TW, rg = tid / TW;
  const bool lane_ok = rg < RG && x < cnt[0] + 2 * HW;
  const int tx = r0[0] + x - HW;
  const unsigned long long mx = g.m[0][x + 3];
  const bool xint = tx >= 1 && tx <= BS - 2;
  const bool xeven = (tx & 1) == 0;
  const int cx = (tx - cb0[0]) >> 1;
  for (int rb = rg; rb < NROW; rb += B * RG) {
    int addr[B], pos[B], cpos[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int r = rb + q * RG;
      addr[q] = self;
      pos[q] = -1;
      cpos[q] = -1;
      const int iy = DIM > 2 ? r % TW : r, iz = DIM > 2 ? r / TW : 0;
      const bool ok = lane_ok && r < NROW && iy < cnt[1] + 2 * HW && (DIM < 3 || iz < cnt[2] + 2 * HW);
      if (!ok) continue;
      const int ty = r0[1] + iy - HW, tz = DIM > 2 ? r0[2] + iz - HW : 0;
      pos[q] = G::idx(x, iy, iz);
      if (HASC && xeven && (ty & 1) == 0 && (tz & 1) == 0)
        cpos[q] = G::cidx(cx, (ty - cb0[1]) >> 1, DIM > 2 ? (tz - cb0[2]) >> 1 : 0);
      const bool inner = xint && ty >= 1 && ty <= BS - 2 && (DIM < 3 || (tz >= 1 && tz <= BS - 2));
      if (inner) {
        addr[q] = self + tx + BS * ty + (DIM > 2 ? BS * BS * tz : 0);
        continue;
      }
      unsigned long long cand = mx & g.m[1][iy + 3];
      if (DIM > 2) cand &= g.m[2][iz + 3];
      if (cand == 0) {  // no holder: predicted later
        pos[q] = -1;
        cpos[q] = -1;
        continue;
      }
      const SEnt E = se[63 - __clzll((long long)cand)];
      addr[q] = E.base + ((2 * tx) >> E.sh) + BS * ((2 * ty) >> E.sh) + (DIM > 2 ? BS * BS * ((2 * tz) >> E.sh) : 0);
    }
    TT v[B][NF];
#pragma unroll
    for (int q = 0; q < B; ++q)
#pragma unroll
      for (int f = 0; f < NF; ++f) v[q][f] = src((size_t)addr[q] + (size_t)f * NP, f);
#pragma unroll
    for (int q = 0; q < B; ++q) {
      if (pos[q] >= 0) {
#pragma unroll
        for (int f = 0; f < NF; ++f) tile[f * TSZ + pos[q]] = v[q][f];
      }
      if (HASC && cpos[q] >= 0) {
#pragma unroll
        for (int f = 0; f < NF; ++f) carr[f * CSZ + cpos[q]] = v[q][f];
      }
    }
  }
  if constexpr (HASC) {
    // coarse-lattice points outside box A, row by row like box A
    constexpr int RGC = NT / CW, NRC = Pow<DIM - 1, CW>::v;
    const int cxl = tid % CW, rgc = tid / CW;
    const int tcx = cb0[0] + 2 * cxl;
    const bool xin = rgc < RGC && tcx <= r0[0] + cnt[0] - 1 + H;
    const bool xa = tcx >= r0[0] - HW && tcx <= r0[0] + cnt[0] - 1 + HW;
    const unsigned long long mcx = xin ? g.m[0][tcx - r0[0] + H] : 0ull;
    for (int rb = rgc; rb < NRC; rb += B * RGC) {
      int addr[B], cpos[B];
#pragma unroll
      for (int q = 0; q < B; ++q) {
        const int r = rb + q * RGC;
        addr[q] = self;
        cpos[q] = -1;
        const int cy = DIM > 2 ? r % CW : r, cz = DIM > 2 ? r / CW : 0;
        const int tcy = cb0[1] + 2 * cy, tcz = DIM > 2 ? cb0[2] + 2 * cz : 0;
        const bool ok = xin && r < NRC && tcy <= r0[1] + cnt[1] - 1 + H &&
                        (DIM < 3 || tcz <= r0[2] + cnt[2] - 1 + H);
        const bool in_a = xa && tcy >= r0[1] - HW && tcy <= r0[1] + cnt[1] - 1 + HW &&
                          (DIM < 3 || (tcz >= r0[2] - HW && tcz <= r0[2] + cnt[2] - 1 + HW));
        if (!ok || in_a) continue;
        unsigned long long cand = mcx & g.m[1][tcy - r0[1] + H];
        if (DIM > 2) cand &= g.m[2][tcz - r0[2] + H];
        if (cand == 0) continue;
        const SEnt E = se[63 - __clzll((long long)cand)];
        addr[q] = E.base + ((2 * tcx) >> E.sh) + BS * ((2 * tcy) >> E.sh) +
                  (DIM > 2 ? BS * BS * ((2 * tcz) >> E.sh) : 0);
        cpos[q] = G::cidx(cxl, cy, cz);
      }
      TT v[B][NF];
#pragma unroll
      for (int q = 0; q < B; ++q)
#pragma unroll
        for (int f = 0; f < NF; ++f) v[q][f] = src((size_t)addr[q] + (size_t)f * NP, f);
#pragma unroll
      for (int q = 0; q < B; ++q)
        if (cpos[q] >= 0) {
#pragma unroll
          for (int f = 0; f < NF; ++f) carr[f * CSZ + cpos[q]] = v[q][f];
        }
    }
  }
  __syncthreads();
}

// Predict the unowned points of box A from the coarse-lattice array, one parity
// class at a time so that a wave's lanes share one unrolled stencil shape.
template <int DIM, int BS, int S, int HW, int NF, typename TT>
struct SPredictBody {
  using G = SGeo<DIM, BS, S, HW>;
  TT* tile;
  const TT* carr;
  const GState<DIM, S + 2 * (HW + 3)>& g;
  const int* r0;
  int a0[3], an[3], cb0[3];
  __device__ __forceinline__ SPredictBody(TT* t_, const TT* c_, const GState<DIM, S + 2 * (HW + 3)>& g_,
                                          const int* r0_, const int* cnt)
      : tile(t_), carr(c_), g(g_), r0(r0_) {
    for (int a = 0; a < 3; ++a) { a0[a] = 0; an[a] = 1; cb0[a] = 0; }
    for (int a = 0; a < DIM; ++a) {
      a0[a] = r0[a] - HW;
      an[a] = cnt[a] + 2 * HW;
      cb0[a] = (r0[a] - G::H + 1) & ~1;
    }
  }
  template <int NX, int NY, int NZ>
  __device__ __forceinline__ void go(int cls) {
    ParityClass<DIM> pc(cls, a0, an);
    for (int p = threadIdx.x; p < pc.total; p += blockDim.x) {
      int t[3];
      pc.coords(p, t);
      bool outside = false;
      for (int a = 0; a < DIM; ++a)
        if (t[a] < 0 || t[a] > BS - 1) outside = true;
      if (!outside) continue;  // the block holds its own points
      int ia[3] = {0, 0, 0};
      unsigned long long cand = ~0ull;
      for (int a = 0; a < DIM; ++a) {
        ia[a] = t[a] - r0[a] + HW;
        cand &= g.m[a][ia[a] + 3];
      }
      if (cand != 0) continue;
      const int bb[3] = {NX == 4 ? (t[0] - 3 - cb0[0]) >> 1 : (t[0] - cb0[0]) >> 1,
                         NY == 4 ? (t[1] - 3 - cb0[1]) >> 1 : (t[1] - cb0[1]) >> 1,
                         DIM > 2 ? (NZ == 4 ? (t[2] - 3 - cb0[2]) >> 1 : (t[2] - cb0[2]) >> 1) : 0};
      const int stride[3] = {1, 1, 1};
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const TT* C = carr + f * G::CSZ;
        auto at = [&](int x, int y, int z) { return C[G::cidx(x, y, z)]; };
        tile[f * G::TSZ + G::idx(ia[0], ia[1], ia[2])] = tensor_fixed<NX, NY, NZ, TT>(at, bb, stride);
      }
    }
  }
};

template <int DIM, int BS, int S, int HW, int NF, typename TT>
__device__ void spredict(TT* tile, const TT* carr, const GState<DIM, S + 2 * (HW + 3)>& g, const int* r0,
                         const int* cnt) {
  SPredictBody<DIM, BS, S, HW, NF, TT> body(tile, carr, g, r0, cnt);
  for_odd_classes<DIM>(body);
  __syncthreads();
}

template <int DIM>
__device__ __forceinline__ void subregion(int sub, int nsub, int S, int BS, int* r0, int* cnt) {
  r0[0] = r0[1] = r0[2] = 0;
  cnt[0] = cnt[1] = cnt[2] = 1;
  for (int a = 0; a < DIM; ++a) {
    const int sa = sub % nsub;
    sub /= nsub;
    r0[a] = sa * S;
    cnt[a] = min(S, BS - r0[a]);
  }
}

// ---------------------------------------------------------------------------
// advection right-hand side at block-local node t (tile coordinates i)
// ---------------------------------------------------------------------------
// (sw: the swirl tables' slices along the region, SWS entries apart; see load_swirl)
// VK: where the velocity comes from -- 0 by ph.kind at run time (the swirl from its
// tables in HBM, or from the LDS slices sw where given), 1 the swirl from the LDS slices
// sw, 2 the constant velocity.  Callers that know the kind pass 1 or 2, so that no
// generic load (an LDS slice or an HBM table) is left in the stencil loop.
template <int DIM, int BS, int S, int H, typename TT, int SWS = S, int VK = 0>
__device__ __forceinline__ TT rhs_adv(const TT* T, const int* i, const int* t, const BlockDesc& d, TT r,
                                      const Physics& ph, const LevelTab& lt, double cfac, const double* sw,
                                      const int* l) {
  using G = Geo<DIM, BS, S, H>;
  const int x = i[0], y = i[1], z = i[2];
  const TT dx = D4(T[G::idx(x - 2, y, z)], T[G::idx(x - 1, y, z)], T[G::idx(x + 1, y, z)], T[G::idx(x + 2, y, z)], r);
  const TT dy = D4(T[G::idx(x, y - 2, z)], T[G::idx(x, y - 1, z)], T[G::idx(x, y + 1, z)], T[G::idx(x, y + 2, z)], r);
  if (VK == 2 || (VK == 0 && ph.kind == 0)) {
    TT acc = (TT)ph.c[0] * dx;
    acc = acc + (TT)ph.c[1] * dy;
    if constexpr (DIM > 2) {
      const TT dz = D4(T[G::idx(x, y, z - 2)], T[G::idx(x, y, z - 1)], T[G::idx(x, y, z + 1)], T[G::idx(x, y, z + 2)], r);
      acc = acc + (TT)ph.c[2] * dz;
    }
    return -acc;
  }
  // swirl: u = sin^2(pi x) sin(2 pi y), v = -sin^2(pi y) sin(2 pi x) from tables on the
  // finest lattice; sw (LDS) holds the region's slices: s2(x), s(x), s2(y), s(y)
  double s2x, sx, s2y, sy;
  if (VK == 1 || sw) {
    s2x = sw[l[0]];
    sx = sw[SWS + l[0]];
    s2y = sw[2 * SWS + l[1]];
    sy = sw[3 * SWS + l[1]];
  } else {
    const int nl = lt.nl[d.level], shift = ph.jmax - d.level;
    int gx = d.c[0] * (BS - 1) + t[0];
    int gy = d.c[1] * (BS - 1) + t[1];
    if (gx >= nl) gx -= nl;
    if (gy >= nl) gy -= nl;
    gx <<= shift;
    gy <<= shift;
    s2x = ph.s2[gx];
    sx = ph.s[gx];
    s2y = ph.s2[gy];
    sy = ph.s[gy];
  }
  const double U = (s2x * sy) * cfac;
  const double W = -((s2y * sx) * cfac);
  return -(((TT)U * dx) + ((TT)W * dy));
}

// swirl table slices of a region into LDS: s2(x), s(x), s2(y), s(y) at its nodes
template <int BS, int S>
__device__ __forceinline__ void load_swirl(double* sw, const BlockDesc& d, const int* r0, const int* cnt,
                                           const StageArgs& A) {
  const int nl = A.lt.nl[d.level], shift = A.ph.jmax - d.level;
  for (int q = threadIdx.x; q < 4 * S; q += blockDim.x) {
    const int k = q / S, l = q % S, ax = k / 2;
    if (l >= cnt[ax]) continue;
    int gg = d.c[ax] * (BS - 1) + r0[ax] + l;
    if (gg >= nl) gg -= nl;
    gg <<= shift;
    sw[q] = (k & 1) ? A.ph.s[gg] : A.ph.s2[gg];
  }
}

// ---------------------------------------------------------------------------
// Navier-Stokes (2D, primitive variables rho, u, v, p): stresses and heat flux
// on [-2, cnt+1]^2 around the region, then the RHS at the region's nodes.
// The tile is FP64.  CT is the arithmetic type: FP64, or FP32 in the mixed form,
// where neighbour differences are still formed in FP64 (exact for close values,
// which FP32 cannot resolve next to a mean flow of O(1)) and everything after the
// difference -- scaling, products, sums, the stress and flux fields -- is FP32.
// ---------------------------------------------------------------------------
template <typename CT>
struct NsConst {
  CT mu, kap, gam, c23, r;
};

// first derivative from four FP64 samples: differences in FP64, the rest in CT
template <typename CT>
__device__ __forceinline__ CT D4d(double um2, double um1, double up1, double up2, CT r) {
  if constexpr (sizeof(CT) == 8) return D4(um2, um1, up1, up2, r);
  else return (8.0f * (CT)(up1 - um1) - (CT)(up2 - um2)) * r;
}

template <int BS, int S, int H, typename CT>
__device__ void ns_fluxes(const double* T, CT* W, const int* cnt, const NsConst<CT>& K) {
  using G = Geo<2, BS, S, H>;
  constexpr int TSZ = G::TSZ, SW = S + 4, SSZ = SW * SW;
  const double* fr = T;
  const double* fu = T + TSZ;
  const double* fv = T + 2 * TSZ;
  const double* fp = T + 3 * TSZ;
  const int nx = cnt[0] + 4, ny = cnt[1] + 4;
  const float rnx = 1.0f / (float)nx;
  for (int p = threadIdx.x; p < nx * ny; p += blockDim.x) {
    const int qy = fdiv(p, rnx);
    const int ux0 = p - qy * nx - 2, uy0 = qy - 2;       // region-local position
    const int x = ux0 + H, y = uy0 + H;                  // tile coordinates
    auto A = [&](const double* F, int xx, int yy) { return F[G::idx(xx, yy, 0)]; };
    auto Tt = [&](int xx, int yy) { return A(fp, xx, yy) / A(fr, xx, yy); };
    const CT ux = D4d<CT>(A(fu, x - 2, y), A(fu, x - 1, y), A(fu, x + 1, y), A(fu, x + 2, y), K.r);
    const CT uy = D4d<CT>(A(fu, x, y - 2), A(fu, x, y - 1), A(fu, x, y + 1), A(fu, x, y + 2), K.r);
    const CT vx = D4d<CT>(A(fv, x - 2, y), A(fv, x - 1, y), A(fv, x + 1, y), A(fv, x + 2, y), K.r);
    const CT vy = D4d<CT>(A(fv, x, y - 2), A(fv, x, y - 1), A(fv, x, y + 1), A(fv, x, y + 2), K.r);
    const CT div = ux + vy;
    const CT tx = D4d<CT>(Tt(x - 2, y), Tt(x - 1, y), Tt(x + 1, y), Tt(x + 2, y), K.r);
    const CT ty = D4d<CT>(Tt(x, y - 2), Tt(x, y - 1), Tt(x, y + 1), Tt(x, y + 2), K.r);
    const int w = (ux0 + 2) + SW * (uy0 + 2);
    W[w] = K.mu * (CT(2) * ux - K.c23 * div);           // tau_xx
    W[SSZ + w] = K.mu * (CT(2) * vy - K.c23 * div);     // tau_yy
    W[2 * SSZ + w] = K.mu * (uy + vx);                  // tau_xy
    W[3 * SSZ + w] = -(K.kap * tx);                     // q_x
    W[4 * SSZ + w] = -(K.kap * ty);                     // q_y
  }
  __syncthreads();
}

template <int BS, int S, int H, typename CT>
__device__ __forceinline__ void ns_rhs(const double* T, const CT* W, int ux0, int uy0, const NsConst<CT>& K, CT* out) {
  using G = Geo<2, BS, S, H>;
  constexpr int TSZ = G::TSZ, SW = S + 4, SSZ = SW * SW;
  const int x = ux0 + H, y = uy0 + H;
  const double* fr = T;
  const double* fu = T + TSZ;
  const double* fv = T + 2 * TSZ;
  const double* fp = T + 3 * TSZ;
  auto A = [&](const double* F, int xx, int yy) { return F[G::idx(xx, yy, 0)]; };
  auto mxx = [&](int xx, int yy) { return A(fr, xx, yy) * A(fu, xx, yy); };
  auto myy = [&](int xx, int yy) { return A(fr, xx, yy) * A(fv, xx, yy); };
  auto Wl = [&](int k, int lx, int ly) { return W[k * SSZ + (lx + 2) + SW * (ly + 2)]; };
  const CT rho = (CT)A(fr, x, y), uu = (CT)A(fu, x, y), vv = (CT)A(fv, x, y), pp = (CT)A(fp, x, y);
  const CT ux = D4d<CT>(A(fu, x - 2, y), A(fu, x - 1, y), A(fu, x + 1, y), A(fu, x + 2, y), K.r);
  const CT uy = D4d<CT>(A(fu, x, y - 2), A(fu, x, y - 1), A(fu, x, y + 1), A(fu, x, y + 2), K.r);
  const CT vx = D4d<CT>(A(fv, x - 2, y), A(fv, x - 1, y), A(fv, x + 1, y), A(fv, x + 2, y), K.r);
  const CT vy = D4d<CT>(A(fv, x, y - 2), A(fv, x, y - 1), A(fv, x, y + 1), A(fv, x, y + 2), K.r);
  const CT px = D4d<CT>(A(fp, x - 2, y), A(fp, x - 1, y), A(fp, x + 1, y), A(fp, x + 2, y), K.r);
  const CT py = D4d<CT>(A(fp, x, y - 2), A(fp, x, y - 1), A(fp, x, y + 1), A(fp, x, y + 2), K.r);
  const CT dmx = D4d<CT>(mxx(x - 2, y), mxx(x - 1, y), mxx(x + 1, y), mxx(x + 2, y), K.r);
  const CT dmy = D4d<CT>(myy(x, y - 2), myy(x, y - 1), myy(x, y + 1), myy(x, y + 2), K.r);
  const CT dtxx = D4(Wl(0, ux0 - 2, uy0), Wl(0, ux0 - 1, uy0), Wl(0, ux0 + 1, uy0), Wl(0, ux0 + 2, uy0), K.r);
  const CT dtxy_y = D4(Wl(2, ux0, uy0 - 2), Wl(2, ux0, uy0 - 1), Wl(2, ux0, uy0 + 1), Wl(2, ux0, uy0 + 2), K.r);
  const CT dtxy_x = D4(Wl(2, ux0 - 2, uy0), Wl(2, ux0 - 1, uy0), Wl(2, ux0 + 1, uy0), Wl(2, ux0 + 2, uy0), K.r);
  const CT dtyy = D4(Wl(1, ux0, uy0 - 2), Wl(1, ux0, uy0 - 1), Wl(1, ux0, uy0 + 1), Wl(1, ux0, uy0 + 2), K.r);
  const CT dqx = D4(Wl(3, ux0 - 2, uy0), Wl(3, ux0 - 1, uy0), Wl(3, ux0 + 1, uy0), Wl(3, ux0 + 2, uy0), K.r);
  const CT dqy = D4(Wl(4, ux0, uy0 - 2), Wl(4, ux0, uy0 - 1), Wl(4, ux0, uy0 + 1), Wl(4, ux0, uy0 + 2), K.r);
  const CT txx = Wl(0, ux0, uy0), tyy = Wl(1, ux0, uy0), txy = Wl(2, ux0, uy0);
  out[0] = -(dmx + dmy);
  out[1] = -(uu * ux + vv * uy) - px / rho + (dtxx + dtxy_y) / rho;
  out[2] = -(uu * vx + vv * vy) - py / rho + (dtxy_x + dtyy) / rho;
  const CT phi = txx * ux + txy * (uy + vx) + tyy * vy;
  const CT divq = dqx + dqy;
  out[3] = -(uu * px + vv * py) - K.gam * pp * (ux + vy) + (K.gam - CT(1)) * (phi - divq);
}

// ---------------------------------------------------------------------------
// fused stage: gather y_s, predict missing ghosts, RHS, store -- one pass over the
// work items of this workgroup; run by the per-stage kernel and by the whole-sweep one
// ---------------------------------------------------------------------------
// what changes from one stage to the next
struct StageVar {
  int stage;              // 1..4
  double alpha;           // y_s = u + alpha k_{s-1}
  const void* kprev;
  void* kout;
  double cfac;            // swirl time factor
};

// static LDS of a stage pass
template <int DIM, int BS, int HW, int NF, int NSUB>
struct StageShared {
  static constexpr int S = (BS + NSUB - 1) / NSUB, H = HW + 3;
  GState<DIM, S + 2 * H> g;
  SEnt se[kMaxEnt];
  double swirl[DIM == 2 && NF == 1 ? 4 * S : 1];
};

template <int DIM, int BS, int HW, int NF, int NSUB, typename TT, typename KT, typename CT, int TPB = 256>
__device__ __forceinline__ void stage_pass(const StageArgs& A, const StageVar& V,
                                           StageShared<DIM, BS, HW, NF, NSUB>& sh, char* smem) {
  constexpr int S = (BS + NSUB - 1) / NSUB, H = HW + 3;
  // rows per lane and gather round: a 3D tile needs ~5 rounds of 8; its occupancy is
  // bound by LDS (3 workgroups per CU), so 10 loads in flight per lane cost nothing
  constexpr int SB = DIM > 2 && NSUB == 1 ? 10 : 8;
  using SG = SGeo<DIM, BS, S, HW>;
  using G = Geo<DIM, BS, S, HW>;  // tile indexing of the right-hand sides
  constexpr int NP = G::NP, TSZ = G::TSZ;
  constexpr int NSUBT = Pow<DIM, NSUB>::v;
  constexpr bool NS = NF == 4;
  static_assert(SG::TSZ == G::TSZ, "tile geometry");
  auto& g = sh.g;
  auto& se = sh.se;
  auto& swirl = sh.swirl;
  TT* tile = reinterpret_cast<TT*>(smem);
  TT* carr = tile + NF * TSZ;
  CT* W = reinterpret_cast<CT*>(carr + NF * SG::CSZ);  // NS stresses / fluxes
  const int nblk = A.topo.h.n_blocks;
  const BlockDesc* blk = A.topo.blk();
  for (XcdWork it(nblk * NSUBT); it.ok(); it.next()) {
    const int w = it.w;
    const int b = A.order ? A.topo.list()[w / NSUBT] : w / NSUBT;
    const BlockDesc d = blk[b];
    int r0[3], cnt[3];
    subregion<DIM>(w % NSUBT, NSUB, S, BS, r0, cnt);
    gsetup<DIM, BS, S, H>(g, d, A.topo.nb(b), A.topo.h.nb_stride, r0);
    sent_setup<DIM, BS, NF>(se, g.ent, d.n_ent);
    const bool sw_lds = DIM == 2 && NF == 1 && A.ph.kind == 1;
    if (sw_lds) load_swirl<BS, S>(swirl, d, r0, cnt, A);
    __syncthreads();
    const bool hasc = d.n_coarse > 0;
    auto gather = [&](const auto& src) {
      if (hasc) sgather<DIM, BS, S, HW, NF, true, TT, SB, TPB>(tile, carr, g, se, d.slot, r0, cnt, src);
      else sgather<DIM, BS, S, HW, NF, false, TT, SB, TPB>(tile, carr, g, se, d.slot, r0, cnt, src);
    };
    if (V.stage == 1) gather(YSrc<TT, KT, false>{A.u, nullptr, 0.0, A.off});
    else gather(YSrc<TT, KT, true>{A.u, (const KT*)V.kprev, V.alpha, A.off});
    if (hasc) spredict<DIM, BS, S, HW, NF, TT>(tile, carr, g, r0, cnt);
    TT r;
    if constexpr (sizeof(TT) == 8) r = A.lt.r[d.level];
    else r = A.lt.rf[d.level];
    const size_t base = (size_t)d.slot * NF * NP;
    const int nn = cnt[0] * cnt[1] * (DIM > 2 ? cnt[2] : 1);
    if constexpr (NS) {
      static_assert(sizeof(TT) == 8, "the NS tile is FP64");
      NsConst<CT> K;
      K.mu = (CT)A.ph.mu;
      K.kap = (CT)A.ph.kap;
      K.gam = (CT)A.ph.gamma;
      K.c23 = (CT)(2.0 / 3.0);
      if constexpr (sizeof(CT) == 8) K.r = A.lt.r[d.level];
      else K.r = A.lt.rf[d.level];
      ns_fluxes<BS, S, HW, CT>(tile, W, cnt, K);
      const float rc0 = 1.0f / (float)cnt[0];
      for (int p = threadIdx.x; p < nn; p += blockDim.x) {
        const int ly = fdiv(p, rc0), lx = p - ly * cnt[0];
        CT kv[4];
        ns_rhs<BS, S, HW, CT>(tile, W, lx, ly, K, kv);
        const int node = (r0[0] + lx) + BS * (r0[1] + ly);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const size_t q = base + (size_t)f * NP + node;
          if (V.stage < 4) {
            ((KT*)V.kout)[q] = (KT)kv[f];
          } else {
            const double k1 = (double)((const KT*)A.k1)[q], k2 = (double)((const KT*)A.k2)[q];
            const double k3 = (double)((const KT*)A.k3)[q], k4 = (double)kv[f];
            A.unew[q] = A.u[q] + A.h6 * ((k1 + k4) + 2.0 * (k2 + k3));
          }
        }
      }
    } else {
      // lanes along x, rows of the region walked by row groups, ER rows per lane and
      // round: the last stage's operands (u, k1, k2, k3) of a round's rows are loaded
      // together, before any of them is used, so their latencies overlap
      constexpr int RGS = TPB / S, NR = Pow<DIM - 1, S>::v;
      constexpr int ER = 4;
      const int lx = (int)threadIdx.x % S, rgs = (int)threadIdx.x / S;
      for (int row0 = rgs; rgs < RGS && lx < cnt[0] && row0 < NR; row0 += ER * RGS) {
        int tq[ER][3];
        bool ok[ER];
        size_t qa[ER];
#pragma unroll
        for (int e = 0; e < ER; ++e) {
          const int row = row0 + e * RGS;
          const int ly = DIM > 2 ? row % S : row, lz = DIM > 2 ? row / S : 0;
          ok[e] = row < NR && ly < cnt[1] && (DIM < 3 || lz < cnt[2]);
          tq[e][0] = r0[0] + lx;
          tq[e][1] = r0[1] + ly;
          tq[e][2] = DIM > 2 ? r0[2] + lz : 0;
          // rows past the region read the block's first node (in bounds) and are dropped
          qa[e] = ok[e] ? base + tq[e][0] + BS * tq[e][1] + (DIM > 2 ? BS * BS * tq[e][2] : 0) : base;
        }
        double e1[ER], e2[ER], e3[ER], eu[ER];
        if (V.stage == 4) {
#pragma unroll
          for (int e = 0; e < ER; ++e) {
            e1[e] = (double)((const KT*)A.k1)[qa[e]];
            e2[e] = (double)((const KT*)A.k2)[qa[e]];
            e3[e] = (double)((const KT*)A.k3)[qa[e]];
            eu[e] = A.u[qa[e]];
          }
        }
#pragma unroll
        for (int e = 0; e < ER; ++e) {
          if (!ok[e]) continue;
          int l[3] = {lx, tq[e][1] - r0[1], DIM > 2 ? tq[e][2] - r0[2] : 0};
          int i[3] = {l[0] + HW, l[1] + HW, DIM > 2 ? l[2] + HW : 0};
          // (one field in 2D: the swirl reads its LDS slices, any other kind is the
          // constant velocity)
          constexpr int VK0 = DIM == 2 && NF == 1 ? 2 : 0;
          const TT kv = sw_lds ? rhs_adv<DIM, BS, S, HW, TT, S, 1>(tile, i, tq[e], d, r, A.ph, A.lt, V.cfac, swirl, l)
                               : rhs_adv<DIM, BS, S, HW, TT, S, VK0>(tile, i, tq[e], d, r, A.ph, A.lt, V.cfac, nullptr, l);
          if (V.stage < 4) {
            ((KT*)V.kout)[qa[e]] = (KT)kv;
          } else {
            const double k4 = (double)kv;
            A.unew[qa[e]] = eu[e] + A.h6 * ((e1[e] + k4) + 2.0 * (e2[e] + e3[e]));
          }
        }
      }
    }
    __syncthreads();
  }
}

template <int DIM, int BS, int HW, int NF, int NSUB, typename TT, typename KT, typename CT, int TPB>
__global__ void __launch_bounds__(TPB) k_stage(StageArgs A) {
  __shared__ StageShared<DIM, BS, HW, NF, NSUB> sh;
  extern __shared__ __align__(16) char smem[];
  stage_pass<DIM, BS, HW, NF, NSUB, TT, KT, CT, TPB>(A, StageVar{A.stage, A.alpha, A.kprev, A.kout, A.cfac}, sh,
                                                     smem);
}

// Grid-wide barrier of the whole-sweep kernel (all workgroups resident: cooperative
// launch).  Arrivals are counted on 8 words (workgroup index mod 8), the last of each
// group counts on a ninth, and the last of those advances the generation word every
// workgroup waits on.  Each arrival releases the workgroup's stores (the last arrival
// of a group acquires them and releases them on with its own count), and one acquire
// fence after the wait makes them visible to the workgroup's next loads; the polls
// themselves are relaxed (an acquiring poll would invalidate the caches each time).
// The wait is bounded: past `spin` polls the workgroup records a time-out and the
// kernel ends (results then void).
__device__ __forceinline__ bool grid_barrier(unsigned* bar, int* err, unsigned spin) {
  __shared__ int ok_sh;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    unsigned* gen = bar + 9 * kBarStride;
    const unsigned g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned* grp = bar + (blockIdx.x & 7) * kBarStride;
    if (__hip_atomic_fetch_add(grp, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) == (gridDim.x >> 3) - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the group's stores, passed on below
      __hip_atomic_store(grp, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      unsigned* top = bar + 8 * kBarStride;
      if (__hip_atomic_fetch_add(top, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == 7u) {
        __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    for (unsigned n = 0; __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0; ++n) {
      if (n >= spin) {
        ok = 0;
        atomicExch(err, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok_sh = ok;
  }
  __syncthreads();
  return ok_sh != 0;
}

// the four stages of an RK4 step in one launch, a grid barrier between stages
template <int DIM, int BS, int HW, int NF, int NSUB, typename TT, typename KT, typename CT>
__global__ void __launch_bounds__(256) k_sweep(SweepArgs S) {
  __shared__ StageShared<DIM, BS, HW, NF, NSUB> sh;
  extern __shared__ __align__(16) char smem[];
  const void* ks[3] = {S.a.k1, S.a.k2, S.a.k3};
  for (int s = 1; s <= 4; ++s) {
    const StageVar V{s, S.alpha[s - 1], s > 1 ? ks[s - 2] : nullptr, s < 4 ? const_cast<void*>(ks[s - 1]) : nullptr,
                     S.cfac[s - 1]};
    stage_pass<DIM, BS, HW, NF, NSUB, TT, KT, CT>(S.a, V, sh, smem);
    if (s < 4 && !grid_barrier(S.bar, S.err, S.spin)) return;
  }
}

// ---------------------------------------------------------------------------
// One-launch RK4 step over overlapped tiles, for 2D advection on a forest whose
// leaves all lie on one level.  There every point a stage reads is held by a
// same-level leaf, and same-level holders compute identical stage values, so a
// workgroup can run its region's four stages alone: it loads u over the region plus
// E points and evaluates k1 on the region + E - HW, k2 on + E - 2 HW, ... -- the halo
// work repeats, with the same operations in the same order, what the neighbours
// compute at their own nodes, so the result is bitwise the four stage launches'.
// k1..k3 stay in LDS; HBM sees u read once and u_new written once.  With ANA the
// halo is 3 points wider, u_new is known up to 3 points beyond the region, and the
// workgroup also runs the analysis of u_new (Sec. 2.3): details, their maxima, the
// flag, and the speculated mothers' nodes, as the analysis kernel does for a forest
// on one level (no finer neighbour, so no redundant node to write back).  A missing
// neighbour (a forest not on one level) yields NaN.
// ---------------------------------------------------------------------------
// A 64-bit value moved between lanes of a row by a DPP pattern (both halves; every lane
// active).
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long x) {
  const unsigned lo = __builtin_amdgcn_update_dpp(0u, (unsigned)x, CTRL, 0xF, 0xF, false);
  const unsigned hi = __builtin_amdgcn_update_dpp(0u, (unsigned)(x >> 32), CTRL, 0xF, 0xF, false);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long lane_u64(unsigned long long x, int lane) {
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)x, lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(x >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}

// Maximum over the 64 lanes of a wave (every lane active) of values that are +0, positive
// or NaN with the sign bit clear (|detail| maxima): as unsigned integers such bit patterns
// order as the values do and every NaN lies above +inf, so the integer maximum is the
// NaN-propagating maximum, without branches.  Within rows of 16 lanes by DPP moves (swap
// neighbours, swap pairs, mirror the half rows, mirror the rows), then the four rows'
// results read out; every lane returns it.
__device__ __forceinline__ double wave_nanmax(double v) {
  unsigned long long u = (unsigned long long)__double_as_longlong(v);
  u = umax64(u, dpp_u64<0xB1>(u));    // quad_perm [1, 0, 3, 2]
  u = umax64(u, dpp_u64<0x4E>(u));    // quad_perm [2, 3, 0, 1]
  u = umax64(u, dpp_u64<0x141>(u));   // row_half_mirror
  u = umax64(u, dpp_u64<0x140>(u));   // row_mirror
  u = umax64(umax64(lane_u64(u, 0), lane_u64(u, 16)), umax64(lane_u64(u, 32), lane_u64(u, 48)));
  return __longlong_as_double((long long)u);
}

// NaN-propagating maxima of two values over a workgroup of TPB threads (values as for
// wave_nanmax): wave maxima through red (2 TPB / 64 doubles of LDS; a barrier must lie
// between two calls), one barrier, then the first wave combines them; only the first
// wave's threads receive the results.
template <int TPB>
__device__ __forceinline__ void wg_nanmax2(double& a, double& b, double* red) {
  a = wave_nanmax(a);
  b = wave_nanmax(b);
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = a;
    red[TPB / 64 + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    a = wave_nanmax(l < TPB / 64 ? red[l] : 0.0);
    b = wave_nanmax(l < TPB / 64 ? red[TPB / 64 + l] : 0.0);
  }
}

template <int BS, int NSUB, bool ANA, bool MA = false>
struct TileGeo {
  // halo: four stages of HW, plus the reach of the details' prediction on the
  // children (3) or on the mothers (6 child nodes)
  static constexpr int HW = 2, E = 4 * HW + (MA ? 6 : (ANA ? 3 : 0));
  static constexpr int S = (BS + NSUB - 1) / NSUB, TW = S + 2 * E, TSZ = TW * TW;
  // slopes are kept where the last stage combines them: the region + E - 4 HW
  static constexpr int KW = S + 2 * (E - 4 * HW), KSZ = KW * KW;
  // LDS bytes: u (FP64), three slope arrays, two stage-value arrays
  template <typename TT, typename KT>
  static constexpr size_t lds() { return (size_t)TSZ * sizeof(double) + 3 * (size_t)KSZ * sizeof(KT) + 2 * (size_t)TSZ * sizeof(TT); }
};

// Every node of [lo, lo + n) in the 2D parity classes C0..3 in one pass, each class on
// waves of its own: class c's q-th node is item base_c + q, where base_c is the previous
// classes' nodes rounded up to whole waves, and item p goes to thread
// (p - rot) mod blockDim.x (a power of two).  So the classes run side by side instead of
// one after another, no wave takes two classes' stencils, and passes that need no barrier
// between them can start on different waves.  body.template at<NX, NY, 1>(t) gets each
// node.
template <int C0, typename B>
__device__ __forceinline__ void for_classes_2d(B& body, const int* lo, const int* n, int rot = 0) {
  int fx[2], nx[2], fy[2], ny[2];   // per axis: first node and count of the even, odd nodes
  for (int odd = 0; odd < 2; ++odd) {
    fx[odd] = lo[0] + (((lo[0] & 1) != odd) ? 1 : 0);
    fy[odd] = lo[1] + (((lo[1] & 1) != odd) ? 1 : 0);
    nx[odd] = fx[odd] <= lo[0] + n[0] - 1 ? (lo[0] + n[0] - 1 - fx[odd]) / 2 + 1 : 0;
    ny[odd] = fy[odd] <= lo[1] + n[1] - 1 ? (lo[1] + n[1] - 1 - fy[odd]) / 2 + 1 : 0;
  }
  int base[5], num[4];
  base[0] = 0;
  for (int c = 0; c < 4; ++c) {
    num[c] = c >= C0 ? nx[c & 1] * ny[c >> 1] : 0;
    base[c + 1] = base[c] + ((num[c] + 63) & ~63);
  }
  // row and column of a class's q-th node by a float reciprocal (q < 2^12 and a row of
  // at most 64 nodes keep (q + 1/2) / n at least 1 / 128 away from an integer, far more
  // than the rounding error, so the truncation is exact)
  const float rx[2] = {1.0f / (float)max(nx[0], 1), 1.0f / (float)max(nx[1], 1)};
  for (int p = (threadIdx.x + rot) & (blockDim.x - 1); p < base[4]; p += blockDim.x) {
    int c = C0;
    while (c < 3 && p >= base[c + 1]) ++c;
    const int q = p - base[c], ox = c & 1, oy = c >> 1;
    if (q >= num[c]) continue;
    const int qy = (int)(((float)q + 0.5f) * rx[ox]);
    const int t[3] = {fx[ox] + 2 * (q - qy * nx[ox]), fy[oy] + 2 * qy, 0};
    if (c == 0) body.template at<1, 1, 1>(t);
    else if (c == 1) body.template at<4, 1, 1>(t);
    else if (c == 2) body.template at<1, 4, 1>(t);
    else body.template at<4, 4, 1>(t);
  }
}

// details of u_new at the region's nodes with an odd coordinate, from the tile's even
// points (stride 2): the analysis kernel's prediction, on the tile's indexing
template <int BS, int S, int E>
struct TileDetails {
  using G = Geo<2, BS, S, E>;
  const double* U;
  const int* r0;
  double* m;
  template <int NX, int NY, int NZ>
  __device__ __forceinline__ void at(const int* t) {
    const int i0 = t[0] - r0[0] + E, i1 = t[1] - r0[1] + E;
    const int bb[3] = {NX == 4 ? i0 - 3 : i0, NY == 4 ? i1 - 3 : i1, 0};
    const int stride[3] = {2, 2, 2};
    auto u = [&](int x, int y, int) { return U[G::idx(x, y, 0)]; };
    const double pred = tensor_fixed<NX, NY, NZ, double>(u, bb, stride);
    m[0] = nanmax(m[0], fabs(U[G::idx(i0, i1, 0)] - pred));
  }
};

// details of the mothers' nodes that lie in the region (a mother node M is the
// child's even node t = 2M - bit (BS-1)): mother-level stencils reach M +- 1, +- 3,
// i.e. child nodes t +- 2, +- 6 (stride 4 in the tile)
template <int BS, int S, int E>
struct MotherDetails {
  using G = Geo<2, BS, S, E>;
  const double* U;
  int off[2], r0[2];
  double* m;
  template <int NX, int NY, int NZ>
  __device__ __forceinline__ void at(const int* M) {
    const int i0 = 2 * M[0] - off[0] - r0[0] + E, i1 = 2 * M[1] - off[1] - r0[1] + E;
    const int bb[3] = {NX == 4 ? i0 - 6 : i0, NY == 4 ? i1 - 6 : i1, 0};
    const int stride[3] = {4, 4, 4};
    auto u = [&](int x, int y, int) { return U[G::idx(x, y, 0)]; };
    const double pred = tensor_fixed<NX, NY, NZ, double>(u, bb, stride);
    m[0] = nanmax(m[0], fabs(U[G::idx(i0, i1, 0)] - pred));
  }
};

template <int BS, int NSUB, typename TT, typename KT, bool ANA, int TPB, bool REF = false, bool MA = false>
__global__ void __launch_bounds__(TPB) k_rk4t(Rk4tArgs A) {
  static_assert(!MA || (ANA && REF), "the mothers' analysis comes with the folded refinement");
  using TG = TileGeo<BS, NSUB, ANA, MA>;
  constexpr int HW = TG::HW, E = TG::E, S = TG::S, TW = TG::TW, TSZ = TG::TSZ, NP = BS * BS;
  constexpr int NSUBT = NSUB * NSUB;
  using G = Geo<2, BS, S, E>;
  static_assert(G::TW == TW, "tile geometry");
  static_assert(S + 2 * (E - HW) <= 64 && (S + 2 * (E - HW)) * (S + 2 * (E - HW)) < 4096,
                "the stage loops' float row split needs rows of at most 64 points, fewer than 2^12 in all");
  constexpr int KW = TG::KW, KSZ = TG::KSZ, KO = E - 4 * HW;   // slope zone: tile index - (E - KO)
  extern __shared__ __align__(16) char smem[];
  double* U = reinterpret_cast<double*>(smem);
  KT* K = reinterpret_cast<KT*>(U + TSZ);          // k1, k2, k3 on the slope zone
  TT* Ya = reinterpret_cast<TT*>(K + 3 * KSZ);     // stage values: this stage's and the next
  TT* Yb = Ya + TSZ;
  __shared__ int tab[9];                            // same-level holder by direction
  __shared__ double sw[4 * TW];
  __shared__ double red[2 * (TPB / 64)];
  const int nblk = A.topo.h.n_blocks;
  const BlockDesc* blk = A.topo.blk();
  const int tid = threadIdx.x;
  for (XcdWork it(nblk * NSUBT); it.ok(); it.next()) {
    const int b = it.w / NSUBT;
    // everything the work item's addresses depend on, requested at once: the block, its
    // (or, with REF, its parent's) entry row up to the row stride -- entries past the
    // count are ignored --, the speculation map and the refinement plan's child slot
    const int ri = b >> 2, ch = b & 3;
    const BlockDesc d = blk[b];
    const BlockDesc P = REF ? A.topo.pblk()[ri] : d;
    const NbEntry* ent = REF ? A.topo.pnb(ri) : A.topo.nb(b);
    const int erow = REF ? A.topo.h.pnb_stride : A.topo.h.nb_stride;
    NbEntry q0;
    if (tid < erow) q0 = ent[tid];
    const int sm = ANA && A.smap ? A.smap[b] : -1;
    const int kslot = REF ? A.topo.ref()[ri].child[ch] : -1;
    int r0[3], cnt[3];
    subregion<2>(it.w % NSUBT, NSUB, S, BS, r0, cnt);
    if (tid < 9) tab[tid] = -1;
    __syncthreads();
    // same-level holders by direction
    auto take = [&](const NbEntry& q) {
      const int ox = q.o[0], oy = q.o[1];
      if (q.dl == 0 && ox % (BS - 1) == 0 && oy % (BS - 1) == 0 && ox >= -(BS - 1) && ox <= BS - 1 &&
          oy >= -(BS - 1) && oy <= BS - 1)
        tab[(oy / (BS - 1) + 1) * 3 + ox / (BS - 1) + 1] = q.slot;
    };
    if (tid < P.n_ent) take(q0);
    for (int e = tid + TPB; e < P.n_ent; e += TPB) take(ent[e]);
    __syncthreads();
    // swirl table slices (first read by the first stage, several barriers on)
    if (A.ph.kind == 1) {
      const int nl = A.lt.nl[d.level], shift = A.ph.jmax - d.level;
      for (int q = tid; q < 4 * TW; q += blockDim.x) {
        const int k = q / TW, l = q % TW, ax = k / 2;
        int gg = d.c[ax] * (BS - 1) + r0[ax] - E + l;
        gg = gg < 0 ? gg + nl : (gg >= nl ? gg - nl : gg);
        gg <<= shift;
        sw[q] = (k & 1) ? A.ph.s[gg] : A.ph.s2[gg];
      }
    }
    // stage values as the stage kernels' gather forms them: y = u + alpha k_{s-1} (in
    // FP64, from the stored slope), minus the field offset in FP32 tiles
    auto stage_value = [&](double y) -> TT {
      if constexpr (sizeof(TT) == 4) return (TT)(y - A.off);
      else return y;
    };
    if constexpr (REF) {
      // The refinement of a forest on one level folded in: the tile is built from the
      // parents.  Block b is child b % 4 of refinement work b / 4 (every parent refines,
      // so children follow their parents in forest order), and a child point takes the
      // synchronised value at the children's level on the parents' grid -- the parent's
      // value at even points, its prediction elsewhere -- as the refinement kernel
      // computes it; the children's pre-step values never reach HBM.
      // Parent-level values over the fine box [r0 + cb - E, r0 + cb + cnt - 1 + E] and
      // the prediction's reach (3 fine points), in the second stage-value array (a
      // quarter of its bytes; unused until the first stage's pass)
      double* PT = reinterpret_cast<double*>(Yb);
      const bool own = kslot == d.slot;
      int cb[2], plo[2], pw[2];
      for (int a = 0; a < 2; ++a) {
        cb[a] = ((ch >> a) & 1) * (BS - 1);
        plo[a] = (r0[a] + cb[a] - E - 3) >> 1;
        pw[a] = ((r0[a] + cb[a] + cnt[a] - 1 + E + 3) >> 1) - plo[a] + 1;
      }
      const float rpw = 1.0f / (float)pw[0];
      for (int p = tid; p < pw[0] * pw[1]; p += blockDim.x) {
        const int qy = fdiv(p, rpw);
        const int px = plo[0] + p - qy * pw[0], py = plo[1] + qy;
        const int dx = px < 0 ? 0 : (px > BS - 1 ? 2 : 1), dy = py < 0 ? 0 : (py > BS - 1 ? 2 : 1);
        const int slot = own ? tab[dy * 3 + dx] : -1;
        const int lx = px - (dx - 1) * (BS - 1), ly = py - (dy - 1) * (BS - 1);
        PT[p] = slot >= 0 ? A.u[(size_t)slot * NP + lx + BS * ly] : __builtin_nan("");
      }
      __syncthreads();
      // the children's values on the fine box, a quad of fine points (2X + {0, 1},
      // 2Y + {0, 1}) per thread: the parent's value, its prediction along x, along y and
      // along both, each as the refinement kernel's per-class tensor stencil forms it (the
      // quad shares the parent values and the x-prediction of row Y)
      int qlo[2], qhi[2], x0[2], nq[2];
      for (int a = 0; a < 2; ++a) {
        qlo[a] = r0[a] + cb[a] - E;
        qhi[a] = qlo[a] + cnt[a] + 2 * E - 1;
        x0[a] = qlo[a] >> 1;
        nq[a] = (qhi[a] >> 1) - x0[a] + 1;
      }
      auto pt = [&](int X, int Y) { return PT[(X - plo[0]) + pw[0] * (Y - plo[1])]; };
      auto put = [&](int qx, int qy, double v) {
        const int i = G::idx(qx - qlo[0], qy - qlo[1], 0);
        U[i] = v;
        Ya[i] = stage_value(v);
      };
      auto row = [&](int X, int Y) { return P4(pt(X - 1, Y), pt(X, Y), pt(X + 1, Y), pt(X + 2, Y)); };
      const float rnq = 1.0f / (float)nq[0];
      for (int p = tid; p < nq[0] * nq[1]; p += blockDim.x) {
        const int qy = fdiv(p, rnq);
        const int X = x0[0] + p - qy * nq[0], Y = x0[1] + qy;
        const bool ex = 2 * X >= qlo[0], ox = 2 * X + 1 <= qhi[0];
        const bool ey = 2 * Y >= qlo[1], oy = 2 * Y + 1 <= qhi[1];
        if (ex && ey) put(2 * X, 2 * Y, pt(X, Y));
        if (ex && oy) put(2 * X, 2 * Y + 1, P4(pt(X, Y - 1), pt(X, Y), pt(X, Y + 1), pt(X, Y + 2)));
        if (ox) {
          const double ry = row(X, Y);
          if (ey) put(2 * X + 1, 2 * Y, ry);
          if (oy) put(2 * X + 1, 2 * Y + 1, P4(row(X, Y - 1), ry, row(X, Y + 1), row(X, Y + 2)));
        }
      }
    } else {
      // u over the region + E
      const int nx = cnt[0] + 2 * E, ny = cnt[1] + 2 * E;
      const float rnx = 1.0f / (float)nx;
      for (int p = tid; p < nx * ny; p += blockDim.x) {
        const int iy = fdiv(p, rnx), ix = p - iy * nx;
        const int tx = r0[0] - E + ix, ty = r0[1] - E + iy;
        const int dx = tx < 0 ? 0 : (tx > BS - 1 ? 2 : 1), dy = ty < 0 ? 0 : (ty > BS - 1 ? 2 : 1);
        const int slot = tab[dy * 3 + dx];
        const int lx = tx - (dx - 1) * (BS - 1), ly = ty - (dy - 1) * (BS - 1);
        const double v = slot >= 0 ? A.u[(size_t)slot * NP + lx + BS * ly] : __builtin_nan("");
        U[G::idx(ix, iy, 0)] = v;
        Ya[G::idx(ix, iy, 0)] = stage_value(v);
      }
    }
    __syncthreads();
    TT r;
    if constexpr (sizeof(TT) == 8) r = A.lt.r[d.level];
    else r = A.lt.rf[d.level];
    TT* Y = Ya;
    TT* Yn = Yb;
    for (int s = 1; s <= 4; ++s) {
      // k_s within E - s HW of the region, and in the same pass the next stage's values
      // there; the last stage forms u_new (in place of u: a point's update reads only
      // its own u) and stores it on the region
      const int mr = E - HW * s;
      const int nx = cnt[0] + 2 * mr, ny = cnt[1] + 2 * mr;
      // row of the p-th point by a float reciprocal (p < 2^12, rows of at most 64
      // points: exact, as in for_classes_2d)
      const float rnx = 1.0f / (float)nx;
      for (int p = tid; p < nx * ny; p += blockDim.x) {
        const int qy = (int)(((float)p + 0.5f) * rnx);
        const int ix = E - mr + (p - qy * nx), iy = E - mr + qy;
        const int i[3] = {ix, iy, 0};
        const int t[3] = {r0[0] - E + ix, r0[1] - E + iy, 0};
        const int l[3] = {ix, iy, 0};
        const int q = G::idx(ix, iy, 0);
        const int kx = ix - (E - KO), ky = iy - (E - KO);
        const bool kz = kx >= 0 && kx < cnt[0] + 2 * KO && ky >= 0 && ky < cnt[1] + 2 * KO;
        const int kq = kx + KW * ky;
        // (the swirl reads its LDS slices, the other kind is the constant velocity)
        const TT kv = A.ph.kind == 1
                          ? rhs_adv<2, BS, S, E, TT, TW, 1>(Y, i, t, d, r, A.ph, A.lt, A.cfac[s - 1], sw, l)
                          : rhs_adv<2, BS, S, E, TT, TW, 2>(Y, i, t, d, r, A.ph, A.lt, A.cfac[s - 1], nullptr, l);
        if (s < 4) {
          const KT ks = (KT)kv;
          if (kz) K[(s - 1) * KSZ + kq] = ks;
          Yn[q] = stage_value(U[q] + A.alpha[s] * (double)ks);
        } else {
          const double k1 = (double)K[kq], k2 = (double)K[KSZ + kq], k3 = (double)K[2 * KSZ + kq];
          const double k4 = (double)kv;
          const double un = U[q] + A.h6 * ((k1 + k4) + 2.0 * (k2 + k3));
          if (ANA) U[q] = un;
          if (t[0] >= r0[0] && t[0] < r0[0] + cnt[0] && t[1] >= r0[1] && t[1] < r0[1] + cnt[1])
            A.unew[(size_t)d.slot * NP + t[0] + BS * t[1]] = un;
        }
      }
      __syncthreads();
      TT* tmp = Y;
      Y = Yn;
      Yn = tmp;
    }
    if constexpr (ANA) {
      // the analysis and the mothers' analysis read u_new only: one pass over both (no
      // barrier between them), then one reduction for both maxima
      double m[1] = {0.0};
      TileDetails<BS, S, E> det{U, r0, m};
      for_classes_2d<1>(det, r0, cnt);
      double mm[1] = {sm >= 0 ? 0.0 : __builtin_nan("")};
      if constexpr (MA) {
        // second analysis of the speculated coarsening: this region's share of its
        // mother's nodes; the host takes the maximum over the shares
        if (sm >= 0) {
          MotherDetails<BS, S, E> md;
          md.U = U;
          md.m = mm;
          int m0[2], mn[2];
          for (int a = 0; a < 2; ++a) {
            md.off[a] = ((sm >> a) & 1) * (BS - 1);
            md.r0[a] = r0[a];
            // mother nodes whose child node lies in [r0, r0 + cnt)
            const int lo = (r0[a] + md.off[a] + 1) >> 1, hi = (r0[a] + cnt[a] - 1 + md.off[a]) >> 1;
            m0[a] = lo;
            mn[a] = hi - lo + 1;
          }
          for_classes_2d<1>(md, m0, mn, (TPB - 384) & (TPB - 1));   // from thread 384 on
        }
      }
      double vb = m[0], vm = mm[0];
      wg_nanmax2<TPB>(vb, vm, red);
      if (tid == 0) {
        if constexpr (NSUBT > 1) {
          A.part[(size_t)b * NSUBT + it.w % NSUBT] = vb;
        } else {
          A.maxd[b] = vb;
          A.flags[b] = d.level > 1 && vb < A.thr ? (int8_t)-1 : (int8_t)0;
        }
        if constexpr (MA) A.mq[(size_t)b * NSUBT + it.w % NSUBT] = vm;
      }
      // speculated coarsening: the mother's nodes this block supplies (every node of a
      // forest on one level is the block's own value); after the reduction, so that no
      // barrier waits for these stores (the next work item rewrites u only after two
      // barriers)
      if (sm >= 0) {
        const int mch = sm & 7;
        const size_t mbase = (size_t)(sm >> 3) * NP;
        ParityClass<2> pc(0, r0, cnt);
        for (int p = (tid + TPB - 576) & (TPB - 1); p < pc.total; p += TPB) {   // from thread 576 on
          int t[3];
          pc.coords(p, t);
          bool skip = false;
          int mnode = 0, mul = 1;
          for (int a = 0; a < 2; ++a) {
            const int bit = (mch >> a) & 1;
            if (bit && t[a] == 0) skip = true;
            mnode += (t[a] / 2 + bit * (BS - 1) / 2) * mul;
            mul *= BS;
          }
          if (!skip) A.unew[mbase + mnode] = U[G::idx(t[0] - r0[0] + E, t[1] - r0[1] + E, 0)];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// plain form: ghost fill into HBM per level, then a separate RHS + update kernel
// ---------------------------------------------------------------------------
template <int DIM, int BS, int HW, int NF>
__global__ void __launch_bounds__(256) k_ghost(StageArgs A) {
  constexpr int H = HW + 3, S = BS;
  using G = Geo<DIM, BS, S, H>;
  constexpr int GW = BS + 2 * HW;
  constexpr int GSZ = Pow<DIM, GW>::v;
  __shared__ GState<DIM, G::TW> g;
  extern __shared__ __align__(16) char smem[];
  double* tile = reinterpret_cast<double*>(smem);
  const int n = A.lvl_end - A.lvl_begin;
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int b = A.topo.list()[A.lvl_begin + w];
    const BlockDesc d = A.topo.blk()[b];
    int r0[3] = {0, 0, 0}, cnt[3] = {BS, DIM > 1 ? BS : 1, DIM > 2 ? BS : 1};
    gsetup<DIM, BS, S, H>(g, d, A.topo.nb(b), A.topo.h.nb_stride, r0);
    const int h_even = d.n_coarse > 0 ? H : 0;
    if (A.stage == 1) {
      YSrc<double, double, false> src{A.u, nullptr, 0.0, A.off};
      gfill<DIM, BS, S, H, NF, double>(tile, g, r0, cnt, HW, h_even, src);
    } else {
      YSrc<double, double, true> src{A.u, (const double*)A.kprev, A.alpha, A.off};
      gfill<DIM, BS, S, H, NF, double>(tile, g, r0, cnt, HW, h_even, src);
    }
    if (d.n_coarse > 0) gpredict<DIM, BS, S, H, NF, double>(tile, g, r0, cnt, HW);
    double* gh = A.ghost + (size_t)d.slot * NF * GSZ;
    for (int p = threadIdx.x; p < NF * GSZ; p += blockDim.x) {
      const int f = p / GSZ, q = p % GSZ;
      const int x = q % GW, y = (q / GW) % GW, z = DIM > 2 ? q / (GW * GW) : 0;
      gh[p] = tile[f * G::TSZ + G::idx(x + 3, y + 3, DIM > 2 ? z + 3 : 0)];
    }
    __syncthreads();
  }
}

// plain form, Navier-Stokes: the ghosted fields from HBM into LDS, then the fused
// form's stresses, fluxes and RHS in FP64
template <int BS, int HW>
__global__ void __launch_bounds__(256) k_rhs_plain_ns(StageArgs A) {
  constexpr int GW = BS + 2 * HW, NP = BS * BS, GSZ = GW * GW;
  using G = Geo<2, BS, BS, HW>;
  static_assert(G::TSZ == GSZ, "ghosted block layout");
  extern __shared__ __align__(16) char smem[];
  double* T = reinterpret_cast<double*>(smem);
  double* W = T + 4 * GSZ;
  const int n = A.lvl_end - A.lvl_begin;
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int b = A.topo.list()[A.lvl_begin + w];
    const BlockDesc d = A.topo.blk()[b];
    const double* gh = A.ghost + (size_t)d.slot * 4 * GSZ;
    for (int p = threadIdx.x; p < 4 * GSZ; p += blockDim.x) T[p] = gh[p];
    __syncthreads();
    NsConst<double> K;
    K.mu = A.ph.mu;
    K.kap = A.ph.kap;
    K.gam = A.ph.gamma;
    K.c23 = 2.0 / 3.0;
    K.r = A.lt.r[d.level];
    const int cnt[3] = {BS, BS, 1};
    ns_fluxes<BS, BS, HW, double>(T, W, cnt, K);
    const size_t base = (size_t)d.slot * 4 * NP;
    for (int p = threadIdx.x; p < NP; p += blockDim.x) {
      double kv[4];
      ns_rhs<BS, BS, HW, double>(T, W, p % BS, p / BS, K, kv);
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const size_t q = base + (size_t)f * NP + p;
        if (A.stage < 4) {
          ((double*)A.kout)[q] = kv[f];
        } else {
          const double k1 = ((const double*)A.k1)[q], k2 = ((const double*)A.k2)[q];
          const double k3 = ((const double*)A.k3)[q], k4 = kv[f];
          A.unew[q] = A.u[q] + A.h6 * ((k1 + k4) + 2.0 * (k2 + k3));
        }
      }
    }
    __syncthreads();
  }
}

template <int DIM, int BS, int HW>
__global__ void __launch_bounds__(256) k_rhs_plain(StageArgs A) {
  constexpr int GW = BS + 2 * HW;
  constexpr int NP = Pow<DIM, BS>::v, GSZ = Pow<DIM, GW>::v;
  using G = Geo<DIM, BS, BS, HW>;
  const int n = A.lvl_end - A.lvl_begin;
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int b = A.topo.list()[A.lvl_begin + w];
    const BlockDesc d = A.topo.blk()[b];
    const double* T = A.ghost + (size_t)d.slot * GSZ;
    const double r = A.lt.r[d.level];
    const size_t base = (size_t)d.slot * NP;
    for (int p = threadIdx.x; p < NP; p += blockDim.x) {
      int t[3] = {p % BS, (p / BS) % BS, DIM > 2 ? p / (BS * BS) : 0};
      int i[3] = {t[0] + HW, t[1] + HW, DIM > 2 ? t[2] + HW : 0};
      const double kv = rhs_adv<DIM, BS, BS, HW, double>(T, i, t, d, r, A.ph, A.lt, A.cfac, nullptr, t);
      if (A.stage < 4) {
        ((double*)A.kout)[base + p] = kv;
      } else {
        const double k1 = ((const double*)A.k1)[base + p];
        const double k2 = ((const double*)A.k2)[base + p];
        const double k3 = ((const double*)A.k3)[base + p];
        A.unew[base + p] = A.u[base + p] + A.h6 * ((k1 + kv) + 2.0 * (k2 + k3));
      }
    }
    (void)G::TSZ;
  }
}

// child nodes of one parity class (see k_refine).  fm[a][i]: finer entries whose region
// holds fine coordinate Q = cb + q0 + i along axis a (null when the parent has no finer
// neighbour); the first such entry in list order supplies a node they hold.
template <int DIM, int BS, int S, int H, int NF, int SQ>
struct RefineBody {
  using G = Geo<DIM, BS, S, H>;
  const double* tile;
  const NbEntry* ent;
  const unsigned long long (*fm)[SQ];
  const int* q0;
  const int* qn;
  const int* r0;
  const int* cb;
  size_t cbase;
  double* u;
  __device__ __forceinline__ RefineBody(const double* t_, const NbEntry* e_, const unsigned long long (*fm_)[SQ],
                                        const int* q0_, const int* qn_, const int* r0_, const int* cb_, size_t cb0,
                                        double* u_)
      : tile(t_), ent(e_), fm(fm_), q0(q0_), qn(qn_), r0(r0_), cb(cb_), cbase(cb0), u(u_) {}
  template <int NX, int NY, int NZ>
  __device__ __forceinline__ void go(int cls) {
    ParityClass<DIM> pc(cls, q0, qn);
    for (int p = threadIdx.x; p < pc.total; p += blockDim.x) {
      int qq[3];
      pc.coords(p, qq);
      int Q[3] = {0, 0, 0};
      bool bnd = false;
      int q = 0, mulq = 1;
      for (int a = 0; a < DIM; ++a) {
        q += qq[a] * mulq;
        mulq *= BS;
        Q[a] = qq[a] + cb[a];
        if (Q[a] == 0 || Q[a] == 2 * (BS - 1)) bnd = true;
      }
      if (cls != 0 && bnd && fm) {
        unsigned long long cand = ~0ull;
        for (int a = 0; a < DIM; ++a) cand &= fm[a][qq[a] - q0[a]];
        if (cand) {
          const NbEntry& E = ent[__ffsll((long long)cand) - 1];
          int s = 0, mul = 1;
          for (int a = 0; a < DIM; ++a) {
            s += (Q[a] - 2 * E.o[a]) * mul;
            mul *= BS;
          }
#pragma unroll
          for (int f = 0; f < NF; ++f) u[cbase + (size_t)f * NP + q] = u[((size_t)E.slot * NF + f) * NP + s];
          continue;
        }
      }
      // parent coordinate -> region-local -> tile coordinate
      const int bb[3] = {NX == 4 ? (Q[0] - 3) / 2 - r0[0] + H : Q[0] / 2 - r0[0] + H,
                         NY == 4 ? (Q[1] - 3) / 2 - r0[1] + H : Q[1] / 2 - r0[1] + H,
                         DIM > 2 ? (NZ == 4 ? (Q[2] - 3) / 2 - r0[2] + H : Q[2] / 2 - r0[2] + H) : 0};
      const int stride[3] = {1, 1, 1};
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double* T = tile + f * TSZ;
        auto at = [&](int x, int y, int z) { return T[G::idx(x, y, z)]; };
        u[cbase + (size_t)f * NP + q] = tensor_fixed<NX, NY, NZ, double>(at, bb, stride);
      }
    }
  }
  static constexpr int TSZ = Geo<DIM, BS, S, H>::TSZ;
  static constexpr int NP = Geo<DIM, BS, S, H>::NP;
};

// ---------------------------------------------------------------------------
// multiresolution analysis: details d = u - P(R(u)), per-field max, flag;
// redundant nodes owned by finer neighbours are written back to the pool
// ---------------------------------------------------------------------------

// details d = u - P(R(u)) of one parity class, the prediction read from the
// coarse-lattice array (its points are the even nodes around the region)
template <int DIM, int BS, int S, int NF>
struct DetailsBodyC {
  using G = SGeo<DIM, BS, S, 0>;
  const double* tile;
  const double* carr;
  const int* r0;
  const int* cnt;
  double* m;
  int cb0[3];
  __device__ __forceinline__ DetailsBodyC(const double* t_, const double* c_, const int* r_, const int* n_, double* m_)
      : tile(t_), carr(c_), r0(r_), cnt(n_), m(m_) {
    for (int a = 0; a < 3; ++a) cb0[a] = a < DIM ? (r0[a] - G::H + 1) & ~1 : 0;
  }
  template <int NX, int NY, int NZ>
  __device__ __forceinline__ void go(int cls) {
    ParityClass<DIM> pc(cls, r0, cnt);
    for (int p = threadIdx.x; p < pc.total; p += blockDim.x) {
      int t[3];
      pc.coords(p, t);
      const int bb[3] = {NX == 4 ? (t[0] - 3 - cb0[0]) >> 1 : (t[0] - cb0[0]) >> 1,
                         NY == 4 ? (t[1] - 3 - cb0[1]) >> 1 : (t[1] - cb0[1]) >> 1,
                         DIM > 2 ? (NZ == 4 ? (t[2] - 3 - cb0[2]) >> 1 : (t[2] - cb0[2]) >> 1) : 0};
      const int stride[3] = {1, 1, 1};
      const int ti = G::idx(t[0] - r0[0], t[1] - r0[1], DIM > 2 ? t[2] - r0[2] : 0);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double* C = carr + f * G::CSZ;
        auto at = [&](int x, int y, int z) { return C[G::cidx(x, y, z)]; };
        const double pred = tensor_fixed<NX, NY, NZ, double>(at, bb, stride);
        m[f] = nanmax(m[f], fabs(tile[f * G::TSZ + ti] - pred));
      }
    }
  }
};

template <int DIM, int BS, int NF, int NSUB, int TPB = 256>
__global__ void __launch_bounds__(TPB) k_mr(MrArgs A) {
  // the region's nodes in the tile; the even nodes up to H = 3 around it (a region may
  // start at an odd node, whose coarse stencil reaches 3 back) in the coarse array
  constexpr int S = (BS + NSUB - 1) / NSUB, H = 3;
  using SG = SGeo<DIM, BS, S, 0>;
  constexpr int NP = SG::NP, TSZ = SG::TSZ;
  constexpr int NSUBT = Pow<DIM, NSUB>::v;
  __shared__ GState<DIM, S + 2 * H> g;
  __shared__ SEnt se[kMaxEnt];
  __shared__ double red[TPB / 64][4];
  extern __shared__ __align__(16) char smem[];
  double* tile = reinterpret_cast<double*>(smem);
  double* carr = tile + NF * TSZ;
  const int nblk = A.topo.h.n_blocks;
  for (XcdWork it(nblk * NSUBT); it.ok(); it.next()) {
    const int w = it.w;
    const int b = w / NSUBT;
    const BlockDesc d = A.topo.blk()[b];
    // speculated coarsening: mother slot * 8 + child index of the block, or -1
    const int sm = A.smap ? A.smap[b] : -1;
    int r0[3], cnt[3];
    subregion<DIM>(w % NSUBT, NSUB, S, BS, r0, cnt);
    gsetup<DIM, BS, S, H>(g, d, A.topo.nb(b), A.topo.h.nb_stride, r0);
    sent_setup<DIM, BS, NF>(se, g.ent, d.n_ent);
    __syncthreads();
    YSrc<double, double, false> src{A.u, nullptr, 0.0, nullptr};
    sgather<DIM, BS, S, 0, NF, true, double, 8, TPB>(tile, carr, g, se, d.slot, r0, cnt, src);
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    const size_t base = (size_t)d.slot * NF * NP;
    const int nn = cnt[0] * cnt[1] * (DIM > 2 ? cnt[2] : 1);
    // redundant nodes owned by a finer neighbour: store the synchronised value
    const float rc0 = 1.0f / (float)cnt[0], rc01 = 1.0f / (float)(cnt[0] * cnt[1]);
    for (int p = threadIdx.x; p < nn; p += blockDim.x) {
      const int q0 = fdiv(p, rc0), q1 = DIM > 2 ? fdiv(p, rc01) : 0;
      const int l[3] = {p - q0 * cnt[0], DIM > 2 ? q0 - q1 * cnt[1] : q0, q1};
      const int t[3] = {r0[0] + l[0], r0[1] + l[1], DIM > 2 ? r0[2] + l[2] : 0};
      bool bnd = false;
      unsigned long long cand = ~0ull;
      for (int a = 0; a < DIM; ++a) {
        if (t[a] == 0 || t[a] == BS - 1) bnd = true;
        cand &= g.m[a][l[a] + H];
      }
      if (bnd && g.ent[63 - __clzll((long long)cand)].dl > 0) {
        const int ti = SG::idx(l[0], l[1], DIM > 2 ? l[2] : 0);
        const int node = t[0] + BS * t[1] + (DIM > 2 ? BS * BS * t[2] : 0);
#pragma unroll
        for (int f = 0; f < NF; ++f) A.u[base + (size_t)f * NP + node] = tile[f * TSZ + ti];
      }
    }
    // details d = u - P(R(u)) at nodes with an odd coordinate (zero at all-even nodes),
    // one parity class at a time so that every lane runs the same unrolled stencil
    DetailsBodyC<DIM, BS, S, NF> det(tile, carr, r0, cnt, m);
    for_odd_classes<DIM>(det);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      double v = m[f];
      for (int off = 32; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off, 64));
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][f] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double v[4];
      for (int f = 0; f < NF; ++f) {
        v[f] = red[0][f];
        for (int q = 1; q < (int)(blockDim.x >> 6); ++q) v[f] = nanmax(v[f], red[q][f]);
      }
      bool last = true;
      if constexpr (NSUBT > 1) {
        // combine sub-tiles: |d| >= 0 (or NaN, whose bit pattern is larger than +Inf), so
        // the unsigned maximum of the bit patterns is the maximum; the last sub-tile to
        // finish reads and clears the partials
        for (int f = 0; f < NF; ++f) atomicMax(&A.acc[(size_t)b * NF + f], (unsigned long long)__double_as_longlong(v[f]));
        __threadfence();
        last = atomicAdd(&A.done[b], 1) == NSUBT - 1;
        if (last) {
          __threadfence();
          for (int f = 0; f < NF; ++f) v[f] = __longlong_as_double((long long)atomicExch(&A.acc[(size_t)b * NF + f], 0ull));
          atomicExch(&A.done[b], 0);
        }
      }
      if (last) {
        bool coarse = d.level > 1;
        for (int f = 0; f < NF; ++f) {
          A.maxd[(size_t)b * NF + f] = v[f];
          if (!(v[f] < A.thr[f])) coarse = false;
        }
        A.flags[b] = coarse ? (int8_t)-1 : (int8_t)0;
      }
    }
    if (sm >= 0) {
      // the block is child `ch` of a speculated family: write the mother's nodes it
      // supplies (R keeps every second node; a node shared by several children comes
      // from the lowest child index), with the values the block holds after the
      // write-back above -- the coarsening kernel's result, without its launch
      const int ch = sm & 7;
      const size_t mbase = (size_t)(sm >> 3) * NF * NP;
      ParityClass<DIM> pc(0, r0, cnt);
      for (int p = threadIdx.x; p < pc.total; p += blockDim.x) {
        int t[3];
        pc.coords(p, t);
        bool skip = false, bnd = false;
        unsigned long long cand = ~0ull;
        int node = 0, mnode = 0, mul = 1;
        for (int a = 0; a < DIM; ++a) {
          const int bit = (ch >> a) & 1;
          if (bit && t[a] == 0) skip = true;
          if (t[a] == 0 || t[a] == BS - 1) bnd = true;
          cand &= g.m[a][t[a] - r0[a] + H];
          node += t[a] * mul;
          mnode += (t[a] / 2 + bit * (BS - 1) / 2) * mul;
          mul *= BS;
        }
        if (skip) continue;
        // interior nodes and nodes written back above: the tile; others: the block's own
        // stored value (a boundary node the tile took from a neighbour)
        const bool from_tile = !bnd || g.ent[63 - __clzll((long long)cand)].dl > 0;
        const int ti = SG::idx(t[0] - r0[0], t[1] - r0[1], DIM > 2 ? t[2] - r0[2] : 0);
#pragma unroll
        for (int f = 0; f < NF; ++f)
          A.u[mbase + (size_t)f * NP + mnode] = from_tile ? tile[f * TSZ + ti] : A.u[base + (size_t)f * NP + node];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// refinement, one workgroup per (parent, child, sub-tile of the child): the
// child's nodes take the synchronised value at level l+1 -- a finer neighbour's
// stored value where one holds the node, else the parent's value (even nodes)
// or its prediction (odd nodes)
// ---------------------------------------------------------------------------
template <int DIM, int BS, int NF, int NSUB>
__global__ void __launch_bounds__(256) k_refine(RefineArgs A) {
  constexpr int SQ = (BS + NSUB - 1) / NSUB;       // child nodes per axis and sub-tile
  constexpr int HWR = 2, H = HWR + 3, S = SQ / 2 + 2;
  using SG = SGeo<DIM, BS, S, HWR>;
  constexpr int NP = SG::NP, NCH = 1 << DIM;
  constexpr int NSUBT = Pow<DIM, NSUB>::v;
  __shared__ GState<DIM, S + 2 * H> g;
  __shared__ SEnt se[kMaxEnt];
  __shared__ unsigned long long fm[DIM][SQ];
  extern __shared__ __align__(16) char smem[];
  double* tile = reinterpret_cast<double*>(smem);
  double* carr = tile + NF * SG::TSZ;
  const int nref = A.topo.h.n_ref;
  for (XcdWork it(nref * NCH * NSUBT); it.ok(); it.next()) {
    const int w = it.w;
    const int ri = w / (NCH * NSUBT), ch = (w / NSUBT) % NCH;
    const RefineDesc R = A.topo.ref()[ri];
    const BlockDesc d = A.topo.pblk()[ri];
    int q0[3], qn[3];
    subregion<DIM>(w % NSUBT, NSUB, SQ, BS, q0, qn);
    // parent region holding the sub-tile's fine nodes Q = cb (bs-1) + q (parent coords Q/2)
    int r0[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
    for (int a = 0; a < DIM; ++a) {
      const int off = ((ch >> a) & 1) * (BS - 1);
      r0[a] = (off + q0[a]) >> 1;
      cnt[a] = ((off + q0[a] + qn[a]) >> 1) - r0[a] + 1;
    }
    gsetup<DIM, BS, S, H>(g, d, A.topo.pnb(ri), A.topo.h.pnb_stride, r0);
    sent_setup<DIM, BS, NF>(se, g.ent, d.n_ent);
    __syncthreads();
    YSrc<double, double, false> src{A.u, nullptr, 0.0, nullptr};
    if (d.n_coarse > 0) {
      sgather<DIM, BS, S, HWR, NF, true, double>(tile, carr, g, se, d.slot, r0, cnt, src);
      spredict<DIM, BS, S, HWR, NF, double>(tile, carr, g, r0, cnt);
    } else {
      sgather<DIM, BS, S, HWR, NF, false, double>(tile, carr, g, se, d.slot, r0, cnt, src);
    }
    const size_t cbase = (size_t)R.child[ch] * NF * NP;
    int cb[3] = {0, 0, 0};
    for (int a = 0; a < DIM; ++a) cb[a] = ((ch >> a) & 1) * (BS - 1);
    // finer entries come last in the list: the lookup table is needed only if the last
    // entry is finer (a uniform branch)
    const bool has_fine = d.n_ent > 0 && g.ent[d.n_ent - 1].dl > 0;
    if (has_fine) {
      for (int k = threadIdx.x; k < DIM * SQ; k += blockDim.x) {
        const int a = k / SQ, i = k % SQ;
        const int Q = cb[a] + q0[a] + i;
        unsigned long long mm = 0;
        for (int e = 0; e < d.n_ent; ++e) {
          const int l = Q - 2 * g.ent[e].o[a];
          if (g.ent[e].dl > 0 && l >= 0 && l <= BS - 1) mm |= 1ull << e;
        }
        fm[a][i] = mm;
      }
      __syncthreads();
    }
    // one parity class of child nodes at a time (fine parity = parity of q, since
    // bs-1 is even): even nodes copy the parent, odd ones are predicted, and nodes on
    // the parent's boundary held by a finer neighbour take that neighbour's value
    RefineBody<DIM, BS, S, HWR, NF, SQ> rf(tile, g.ent, has_fine ? fm : nullptr, q0, qn, r0, cb, cbase, A.u);
    rf.template go<1, 1, 1>(0);
    for_odd_classes<DIM>(rf);
    __syncthreads();
  }
}

// coarsening: the mother keeps every second node of her children (restriction R);
// a node shared by several children is taken from the lowest child index
template <int DIM, int BS, int NF>
__global__ void __launch_bounds__(256) k_coarsen(CoarsenArgs A) {
  constexpr int NP = Pow<DIM, BS>::v;
  const int nfam = A.topo.h.n_fam;
  const long total = (long)nfam * NP;
  const FamilyDesc* fam = A.topo.fam();
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < total; p += (long)gridDim.x * blockDim.x) {
    const int fi = (int)(p / NP), q = (int)(p % NP);
    const FamilyDesc& F = fam[fi];
    int ii[3] = {q % BS, (q / BS) % BS, DIM > 2 ? q / (BS * BS) : 0};
    int ch = 0, s = 0, mul = 1;
    for (int a = 0; a < DIM; ++a) {
      const int bit = 2 * ii[a] > BS - 1 ? 1 : 0;
      ch |= bit << a;
      s += (2 * ii[a] - bit * (BS - 1)) * mul;
      mul *= BS;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f)
      A.u[((size_t)F.parent * NF + f) * NP + q] = A.u[((size_t)F.child[ch] * NF + f) * NP + s];
  }
}

// ---------------------------------------------------------------------------
// shock-capturing filter after a time step (Navier-Stokes, 2D, whole blocks): per
// axis a pressure sensor s = max(0, 1 - r_th / r) with r = M / p^2 + 1e-16,
// M = ((Dp_j - Dp_{j+1})^2 + (Dp_j - Dp_{j-1})^2) / 2, Dp_j = (-p_{j+1} + 2 p_j - p_{j-1}) / 4,
// switches a second-order filter in flux form on every field:
// q_i - [(s_{i+1/2} F_{i+1/2} - s_{i-1/2} F_{i-1/2})_x + (...)_y], s_{i+1/2} = (s_i + s_{i+1}) / 2,
// F_{i+1/2} = -(q_{i+1} - q_i) / 4, on the synchronised state; written to unew
// ---------------------------------------------------------------------------
template <int BS, int NF>
__global__ void __launch_bounds__(256) k_filter(FilterArgs A) {
  constexpr int HW = 4, S = BS, H = HW + 3, SW = BS + 2;
  using SG = SGeo<2, BS, S, HW>;
  constexpr int TSZ = SG::TSZ, NP = SG::NP;
  __shared__ GState<2, S + 2 * H> g;
  __shared__ SEnt se[kMaxEnt];
  extern __shared__ __align__(16) char smem[];
  double* tile = reinterpret_cast<double*>(smem);
  double* carr = tile + NF * TSZ;
  double* sx = carr + NF * SG::CSZ;   // sensor along x at x = -1..BS, y = 0..BS-1
  double* sy = sx + SW * BS;          // sensor along y at x = 0..BS-1, y = -1..BS
  const double rth = A.rth;
  const int nblk = A.topo.h.n_blocks;
  for (XcdWork it(nblk); it.ok(); it.next()) {
    const int b = it.w;
    const BlockDesc d = A.topo.blk()[b];
    int r0[3] = {0, 0, 0}, cnt[3] = {BS, BS, 1};
    gsetup<2, BS, S, H>(g, d, A.topo.nb(b), A.topo.h.nb_stride, r0);
    sent_setup<2, BS, NF>(se, g.ent, d.n_ent);
    __syncthreads();
    YSrc<double, double, false> src{A.u, nullptr, 0.0, nullptr};
    if (d.n_coarse > 0) {
      sgather<2, BS, S, HW, NF, true, double>(tile, carr, g, se, d.slot, r0, cnt, src);
      spredict<2, BS, S, HW, NF, double>(tile, carr, g, r0, cnt);
    } else {
      sgather<2, BS, S, HW, NF, false, double>(tile, carr, g, se, d.slot, r0, cnt, src);
    }
    auto Q = [&](int f, int x, int y) { return tile[f * TSZ + SG::idx(x + HW, y + HW, 0)]; };
    auto sens = [&](int x, int y, int ax) -> double {
      auto P = [&](int dd) { return ax == 0 ? Q(NF - 1, x + dd, y) : Q(NF - 1, x, y + dd); };
      auto Dp = [&](int dd) { return ((-P(dd + 1) + 2.0 * P(dd)) - P(dd - 1)) * 0.25; };
      const double d0 = Dp(0), dp = Dp(1), dm = Dp(-1);
      const double m = ((d0 - dp) * (d0 - dp) + (d0 - dm) * (d0 - dm)) * 0.5;
      const double p0 = P(0);
      const double r = m / (p0 * p0) + 1e-16;
      const double sv = 1.0 - rth / r;
      return sv > 0.0 ? sv : 0.0;
    };
    for (int p = threadIdx.x; p < SW * BS; p += blockDim.x) {
      sx[p] = sens(p % SW - 1, p / SW, 0);
      sy[p] = sens(p % BS, p / BS - 1, 1);
    }
    __syncthreads();
    const size_t base = (size_t)d.slot * NF * NP;
    for (int p = threadIdx.x; p < BS * BS; p += blockDim.x) {
      const int x = p % BS, y = p / BS;
      const double sx0 = sx[(x + 1) + SW * y], sy0 = sy[x + BS * (y + 1)];
      const double sxm = (sx[x + SW * y] + sx0) * 0.5, sxp = (sx0 + sx[(x + 2) + SW * y]) * 0.5;
      const double sym = (sy[x + BS * y] + sy0) * 0.5, syp = (sy0 + sy[x + BS * (y + 2)]) * 0.5;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double q = Q(f, x, y);
        const double fxp = -(Q(f, x + 1, y) - q) * 0.25, fxm = -(q - Q(f, x - 1, y)) * 0.25;
        const double fyp = -(Q(f, x, y + 1) - q) * 0.25, fym = -(q - Q(f, x, y - 1)) * 0.25;
        A.unew[base + (size_t)f * NP + x + BS * y] = q - ((sxp * fxp - sxm * fxm) + (syp * fyp - sym * fym));
      }
    }
    __syncthreads();
  }
}

// read-back of synchronised block values in forest order
template <int DIM, int BS, int NF>
__global__ void __launch_bounds__(256) k_read(ReadArgs A) {
  constexpr int H = 0, S = BS;
  using G = Geo<DIM, BS, S, H>;
  constexpr int NP = G::NP;
  __shared__ GState<DIM, G::TW> g;
  extern __shared__ __align__(16) char smem[];
  double* tile = reinterpret_cast<double*>(smem);
  const int nblk = A.topo.h.n_blocks;
  for (XcdWork it(nblk); it.ok(); it.next()) {
    const int b = it.w;
    const BlockDesc d = A.topo.blk()[b];
    int r0[3] = {0, 0, 0}, cnt[3] = {BS, BS, DIM > 2 ? BS : 1};
    gsetup<DIM, BS, S, H>(g, d, A.topo.nb(b), A.topo.h.nb_stride, r0);
    YSrc<double, double, false> src{A.u, nullptr, 0.0, nullptr};
    gfill<DIM, BS, S, H, NF, double>(tile, g, r0, cnt, 0, 0, src);
    if (A.level == 0) {
      for (int p = threadIdx.x; p < NF * NP; p += blockDim.x) A.out[(size_t)b * NF * NP + p] = tile[p];
    } else {
      // nodes on the level-L lattice go to their place in the uniform array; nodes
      // shared with neighbours hold the same synchronised value in every holder
      const int sh = d.level - A.level;
      const long nl = (long)(1L << A.level) * (BS - 1);
      const long ntot = DIM > 2 ? nl * nl * nl : nl * nl;
      for (int p = threadIdx.x; p < NP; p += blockDim.x) {
        const int t[3] = {p % BS, DIM > 2 ? (p / BS) % BS : p / BS, DIM > 2 ? p / (BS * BS) : 0};
        long m = 0, mul = 1;
        bool on = true;
        for (int a = 0; a < DIM; ++a) {
          const long gq = (long)d.c[a] * (BS - 1) + t[a];
          if (gq & ((1L << sh) - 1)) on = false;
          m += ((gq >> sh) % nl) * mul;
          mul *= nl;
        }
        if (!on) continue;
#pragma unroll
        for (int f = 0; f < NF; ++f) A.out[(size_t)f * ntot + m] = tile[f * NP + p];
      }
    }
    __syncthreads();
  }
}

// whole-block copy from a contiguous [n][bsz] array into pool slots
__global__ void __launch_bounds__(256) k_scatter(const double* src, const int* slots, int n, size_t bsz, double* dst) {
  const size_t total = (size_t)n * bsz;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < total; p += (size_t)gridDim.x * blockDim.x) {
    const size_t b = p / bsz, q = p % bsz;
    dst[(size_t)slots[b] * bsz + q] = src[p];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename K, typename Arg>
static hipError_t go(K kern, int grid, size_t lds, hipStream_t st, const Arg& a, int threads = 256) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  grid = ((grid > 0 ? grid : 1) + 7) & ~7;  // XcdWork needs a multiple of 8
  hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, st, a);
  return hipGetLastError();
}

// TT: tile type, KT: slope storage type, CT: arithmetic type, TPB: threads per workgroup
template <int DIM, int BS, int HW, int NF, int NSUB, typename TT, typename KT, typename CT, int TPB>
static hipError_t stage_go(int grid, const StageArgs& a, hipStream_t st) {
  constexpr int S = (BS + NSUB - 1) / NSUB;
  using SG = SGeo<DIM, BS, S, HW>;
  size_t lds = sizeof(TT) * NF * (SG::TSZ + SG::CSZ);
  if (NF == 4) lds += sizeof(CT) * 5 * (S + 4) * (S + 4);
  return go(k_stage<DIM, BS, HW, NF, NSUB, TT, KT, CT, TPB>, grid, lds, st, a, TPB);
}

// whole sweep: the grid is what the device holds at once (all workgroups must be
// resident for the grid barrier), capped by the work; a multiple of 8 (XcdWork and
// the barrier's 8 arrival groups)
template <int DIM, int BS, int HW, int NF, int NSUB, typename TT, typename KT, typename CT>
static hipError_t sweep_go(int max_grid, const SweepArgs& a, hipStream_t st, int* grid_out) {
  constexpr int S = (BS + NSUB - 1) / NSUB;
  using SG = SGeo<DIM, BS, S, HW>;
  size_t lds = sizeof(TT) * NF * (SG::TSZ + SG::CSZ);
  if (NF == 4) lds += sizeof(CT) * 5 * (S + 4) * (S + 4);
  auto kern = k_sweep<DIM, BS, HW, NF, NSUB, TT, KT, CT>;
  static int resident = 0, cus = 0;   // per instantiation (one device per process)
  if (!resident) {
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    int dev = 0, per_cu = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, 256, lds);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    resident = per_cu * ncu;
    cus = ncu;
  }
  // at most one workgroup per compute unit: each barrier costs a release and an
  // acquire per workgroup, so fewer, busier workgroups pay less for it
  int grid = std::min(std::min(resident, cus), std::max(max_grid, 8));
  grid &= ~7;
  if (grid < 8) return hipErrorInvalidConfiguration;
  *grid_out = grid;
  SweepArgs arg = a;
  void* params[] = {&arg};
  return hipLaunchCooperativeKernel((const void*)kern, dim3(grid), dim3(256), params, (unsigned)lds, st);
}

// FP64: FP64 tile, slopes and arithmetic.  Mixed: FP32 slopes and arithmetic; the
// tile is FP32 (stage values minus a per-field offset) for advection and FP64 for
// Navier-Stokes (neighbour differences formed in FP64, see ns_fluxes).
template <int D, int B, int W, int F, int NS, int P, int T>
static hipError_t stage_pick(int grid, const StageArgs& a, hipStream_t st) {
  if constexpr (P == 0) return stage_go<D, B, W, F, NS, double, double, double, T>(grid, a, st);
  else if constexpr (F == 4) return stage_go<D, B, W, F, NS, double, float, float, T>(grid, a, st);
  else return stage_go<D, B, W, F, NS, float, float, float, T>(grid, a, st);
}

template <int D, int B, int W, int F, int NS, int P>
static hipError_t sweep_pick(int max_grid, const SweepArgs& a, hipStream_t st, int* grid_out) {
  if constexpr (P == 0) return sweep_go<D, B, W, F, NS, double, double, double>(max_grid, a, st, grid_out);
  else if constexpr (F == 4) return sweep_go<D, B, W, F, NS, double, float, float>(max_grid, a, st, grid_out);
  else return sweep_go<D, B, W, F, NS, float, float, float>(max_grid, a, st, grid_out);
}

// compiled stage variants: shape, precision (0 FP64, 1 mixed), sub-tiles per axis,
// threads per workgroup (512 only where a sub-tile has enough points for them)
#define MRB_STAGE_VARIANTS(X) \
  X(2, 17, 2, 1, 0, 1, 256)   \
  X(2, 17, 2, 1, 0, 2, 256)   \
  X(2, 17, 2, 1, 1, 1, 256)   \
  X(2, 17, 2, 1, 1, 2, 256)   \
  X(2, 33, 2, 1, 0, 1, 256)   \
  X(2, 33, 2, 1, 0, 1, 512)   \
  X(2, 33, 2, 1, 0, 2, 256)   \
  X(2, 33, 2, 1, 0, 4, 256)   \
  X(2, 33, 2, 1, 1, 1, 256)   \
  X(2, 33, 2, 1, 1, 1, 512)   \
  X(2, 33, 2, 1, 1, 2, 256)   \
  X(2, 33, 2, 1, 1, 4, 256)   \
  X(2, 33, 4, 4, 0, 2, 256)   \
  X(2, 33, 4, 4, 0, 2, 512)   \
  X(2, 33, 4, 4, 0, 4, 256)   \
  X(2, 33, 4, 4, 1, 1, 256)   \
  X(2, 33, 4, 4, 1, 1, 512)   \
  X(2, 33, 4, 4, 1, 1, 1024)  \
  X(2, 33, 4, 4, 1, 2, 256)   \
  X(2, 33, 4, 4, 1, 2, 512)   \
  X(2, 33, 4, 4, 1, 4, 256)   \
  X(3, 17, 2, 1, 0, 2, 256)   \
  X(3, 17, 2, 1, 0, 2, 512)   \
  X(3, 17, 2, 1, 1, 1, 256)   \
  X(3, 17, 2, 1, 1, 1, 512)   \
  X(3, 17, 2, 1, 1, 2, 256)   \
  X(3, 17, 2, 1, 1, 2, 512)

#define MRB_SHAPES(X) \
  X(2, 17, 2, 1)      \
  X(2, 33, 2, 1)      \
  X(2, 33, 4, 4)      \
  X(3, 17, 2, 1)

bool shape_supported(const Shape& s) {
#define X(D, B, W, F) if (s.dim == D && s.bs == B && s.hw == W && s.nf == F) return true;
  MRB_SHAPES(X)
#undef X
  return false;
}

int stage_variants(const Shape& s, int precision, int* nsub, int cap) {
  int n = 0;
#define X(D, B, W, F, P, NS, T)                                                                  \
  if (s.dim == D && s.bs == B && s.hw == W && s.nf == F && precision == P && T == 256 && n < cap) \
    nsub[n++] = NS;
  MRB_STAGE_VARIANTS(X)
#undef X
  return n;
}

int stage_threads(const Shape& s, int precision, int nsub, int* tpb, int cap) {
  int n = 0;
#define X(D, B, W, F, P, NS, T) \
  if (s.dim == D && s.bs == B && s.hw == W && s.nf == F && precision == P && NS == nsub && n < cap) tpb[n++] = T;
  MRB_STAGE_VARIANTS(X)
#undef X
  return n;
}

hipError_t launch_stage(const Shape& s, int precision, Variant v, int grid, const StageArgs& a, hipStream_t st) {
#define X(D, B, W, F, P, NS, T)                                                                  \
  if (s.dim == D && s.bs == B && s.hw == W && s.nf == F && precision == P && v.nsub == NS &&     \
      v.tpb == T)                                                                                \
    return stage_pick<D, B, W, F, NS, P, T>(grid, a, st);
  MRB_STAGE_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

// overlapped-tile RK4 variants: shape (2D, one field, halo 2), precision, sub-tiles per axis
#define MRB_RK4T_VARIANTS(X) \
  X(17, 0, 1) X(17, 1, 1)    \
  X(33, 0, 1) X(33, 0, 2) X(33, 0, 4) X(33, 1, 1) X(33, 1, 2) X(33, 1, 4)

// with the analysis folded in, whole blocks and quarters may take 512 or 1024 threads (a
// forest small enough for this form leaves most compute units idle otherwise)
template <int B, int NS, typename TT, typename KT>
static hipError_t rk4t_go(bool ana, bool ref, bool ma, int tpb, int grid, const Rk4tArgs& a, hipStream_t st) {
  if (ma) {
    if (!ana || !ref) return hipErrorInvalidValue;
    const size_t lds = TileGeo<B, NS, true, true>::template lds<TT, KT>();
    if (tpb == 256) return go(k_rk4t<B, NS, TT, KT, true, 256, true, true>, grid, lds, st, a, 256);
    if constexpr (NS <= 2) {
      if (tpb == 512) return go(k_rk4t<B, NS, TT, KT, true, 512, true, true>, grid, lds, st, a, 512);
      if (tpb == 1024) return go(k_rk4t<B, NS, TT, KT, true, 1024, true, true>, grid, lds, st, a, 1024);
    }
    return hipErrorInvalidValue;
  }
  if (ana) {
    const size_t lds = TileGeo<B, NS, true>::template lds<TT, KT>();
    if (ref) {
      if (tpb == 256) return go(k_rk4t<B, NS, TT, KT, true, 256, true>, grid, lds, st, a, 256);
      if constexpr (NS <= 2) {
        if (tpb == 512) return go(k_rk4t<B, NS, TT, KT, true, 512, true>, grid, lds, st, a, 512);
        if (tpb == 1024) return go(k_rk4t<B, NS, TT, KT, true, 1024, true>, grid, lds, st, a, 1024);
      }
      return hipErrorInvalidValue;
    }
    if (tpb == 256) return go(k_rk4t<B, NS, TT, KT, true, 256>, grid, lds, st, a, 256);
    if constexpr (NS <= 2) {
      if (tpb == 512) return go(k_rk4t<B, NS, TT, KT, true, 512>, grid, lds, st, a, 512);
      if (tpb == 1024) return go(k_rk4t<B, NS, TT, KT, true, 1024>, grid, lds, st, a, 1024);
    }
    return hipErrorInvalidValue;
  }
  if (ref) return hipErrorInvalidValue;
  if (tpb != 256) return hipErrorInvalidValue;
  return go(k_rk4t<B, NS, TT, KT, false, 256>, grid, TileGeo<B, NS, false>::template lds<TT, KT>(), st, a);
}

hipError_t launch_rk4t(const Shape& s, int precision, int nsub, bool analysis, bool refine, bool mothers, int tpb,
                       int grid, const Rk4tArgs& a, hipStream_t st) {
  if (s.dim != 2 || s.hw != 2 || s.nf != 1) return hipErrorInvalidValue;
#define X(B, P, NS)                                                                                              \
  if (s.bs == B && precision == P && nsub == NS) {                                                              \
    if constexpr (P == 0) return rk4t_go<B, NS, double, double>(analysis, refine, mothers, tpb, grid, a, st);   \
    else return rk4t_go<B, NS, float, float>(analysis, refine, mothers, tpb, grid, a, st);                      \
  }
  MRB_RK4T_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

int rk4t_variants(const Shape& s, int precision, int* nsub, int cap) {
  int n = 0;
  if (s.dim != 2 || s.hw != 2 || s.nf != 1) return 0;
#define X(B, P, NS) if (s.bs == B && precision == P && n < cap) nsub[n++] = NS;
  MRB_RK4T_VARIANTS(X)
#undef X
  return n;
}

hipError_t launch_sweep(const Shape& s, int precision, Variant v, int max_grid, const SweepArgs& a, hipStream_t st,
                        int* grid_out) {
#define X(D, B, W, F, P, NS, T)                                                                  \
  if (s.dim == D && s.bs == B && s.hw == W && s.nf == F && precision == P && v.nsub == NS && T == 256) \
    return sweep_pick<D, B, W, F, NS, P>(max_grid, a, st, grid_out);
  MRB_STAGE_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

template <int DIM, int BS, int HW, int NF>
static hipError_t plain_go(int grid, const StageArgs& a, hipStream_t st) {
  using G = Geo<DIM, BS, BS, HW + 3>;
  hipError_t e = go(k_ghost<DIM, BS, HW, NF>, grid, sizeof(double) * NF * G::TSZ, st, a);
  if (e != hipSuccess) return e;
  if constexpr (NF == 4) {
    constexpr int GW = BS + 2 * HW;
    return go(k_rhs_plain_ns<BS, HW>, grid, sizeof(double) * (4 * GW * GW + 5 * (BS + 4) * (BS + 4)), st, a);
  } else {
    return go(k_rhs_plain<DIM, BS, HW>, grid, 0, st, a);
  }
}

hipError_t launch_plain(const Shape& s, int grid, const StageArgs& a, hipStream_t st) {
#define X(D, B, W, F) if (s.dim == D && s.bs == B && s.hw == W && s.nf == F) return plain_go<D, B, W, F>(grid, a, st);
  MRB_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

// analysis (kind 0) and refinement (kind 1) tilings per shape
#define MRB_AUX_VARIANTS(X) \
  X(2, 17, 2, 1, 1)         \
  X(2, 17, 2, 1, 2)         \
  X(2, 33, 2, 1, 1)         \
  X(2, 33, 2, 1, 2)         \
  X(2, 33, 2, 1, 4)         \
  X(2, 33, 4, 4, 1)         \
  X(2, 33, 4, 4, 2)         \
  X(3, 17, 2, 1, 1)         \
  X(3, 17, 2, 1, 2)

int aux_variants(const Shape& s, int kind, int* nsub, int cap) {
  int n = 0;
  (void)kind;
#define X(D, B, W, F, NS) if (s.dim == D && s.bs == B && s.hw == W && s.nf == F && n < cap) nsub[n++] = NS;
  MRB_AUX_VARIANTS(X)
#undef X
  return n;
}

template <int D, int B, int F, int NS, int T = 256>
static hipError_t mr_go(int grid, const MrArgs& a, hipStream_t st) {
  constexpr int S = (B + NS - 1) / NS;
  using SG = SGeo<D, B, S, 0>;
  return go(k_mr<D, B, F, NS, T>, grid, sizeof(double) * F * (SG::TSZ + SG::CSZ), st, a, T);
}

// the analysis of whole 2D blocks with larger workgroups (a small forest leaves most
// compute units idle with 256 threads per block): shape, threads per workgroup
#define MRB_MR_WIDE(X) \
  X(2, 33, 2, 1, 512)  \
  X(2, 33, 2, 1, 1024) \
  X(2, 33, 4, 4, 512)  \
  X(2, 33, 4, 4, 1024)

int mr_threads(const Shape& s, int nsub, int* tpb, int cap) {
  int n = 0;
  if (cap > 0) tpb[n++] = 256;
  if (nsub != 1) return n;
#define X(D, B, W, F, T) if (s.dim == D && s.bs == B && s.hw == W && s.nf == F && n < cap) tpb[n++] = T;
  MRB_MR_WIDE(X)
#undef X
  return n;
}

template <int D, int B, int F, int NS>
static hipError_t refine_go(int grid, const RefineArgs& a, hipStream_t st) {
  constexpr int SQ = (B + NS - 1) / NS;
  using SG = SGeo<D, B, SQ / 2 + 2, 2>;
  return go(k_refine<D, B, F, NS>, grid, sizeof(double) * F * (SG::TSZ + SG::CSZ), st, a);
}

hipError_t launch_mr(const Shape& s, int nsub, int tpb, int grid, const MrArgs& a, hipStream_t st) {
  if (tpb != 256) {
#define X(D, B, W, F, T) \
    if (s.dim == D && s.bs == B && s.hw == W && s.nf == F && nsub == 1 && tpb == T) return mr_go<D, B, F, 1, T>(grid, a, st);
    MRB_MR_WIDE(X)
#undef X
    return hipErrorInvalidValue;
  }
#define X(D, B, W, F, NS) \
  if (s.dim == D && s.bs == B && s.hw == W && s.nf == F && nsub == NS) return mr_go<D, B, F, NS>(grid, a, st);
  MRB_AUX_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_refine(const Shape& s, int nsub, int grid, const RefineArgs& a, hipStream_t st) {
#define X(D, B, W, F, NS) \
  if (s.dim == D && s.bs == B && s.hw == W && s.nf == F && nsub == NS) return refine_go<D, B, F, NS>(grid, a, st);
  MRB_AUX_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_coarsen(const Shape& s, int grid, const CoarsenArgs& a, hipStream_t st) {
#define X(D, B, W, F) if (s.dim == D && s.bs == B && s.hw == W && s.nf == F) return go(k_coarsen<D, B, F>, grid, 0, st, a);
  MRB_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_read(const Shape& s, int grid, const ReadArgs& a, hipStream_t st) {
#define X(D, B, W, F)                                                                   \
  if (s.dim == D && s.bs == B && s.hw == W && s.nf == F)                                \
    return go(k_read<D, B, F>, grid, sizeof(double) * F * Geo<D, B, B, 0>::TSZ, st, a);
  MRB_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Library-owned scratch for the entry point that allocates nothing (the analysis
// with sub-tiled workgroups: per-block partial maxima and completion counters).
// Every GPU the library runs on holds one copy of this array until the process ends,
// shared by every call on that GPU.  Host code never passes the array's name to a
// kernel: it looks up the device address once per device and passes that.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_addr[kMaxDevices];
}  // namespace

hipError_t scratch_setup(void** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(scratch_mu);
  if (!scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_addr[dev] = p;
  }
  *out = scratch_addr[dev];
  return hipSuccess;
}

// zero fill (used instead of hipMemsetAsync where a caller may capture the work)
__global__ void __launch_bounds__(256) k_zero(unsigned* p, size_t nwords) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t nw = bytes / sizeof(unsigned);
  if (nw == 0) return hipSuccess;
  const int grid = (int)std::min<size_t>((nw + 255) / 256, 1024);
  hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, st, (unsigned*)p, nw);
  return hipGetLastError();
}

hipError_t launch_filter(const Shape& s, int grid, const FilterArgs& a, hipStream_t st) {
  if (s.dim == 2 && s.bs == 33 && s.hw == 4 && s.nf == 4) {
    using SG = SGeo<2, 33, 33, 4>;
    const size_t lds = sizeof(double) * (4 * (SG::TSZ + SG::CSZ) + 2 * 35 * 33);
    return go(k_filter<33, 4>, grid, lds, st, a);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_scatter(const double* src, const int* slots, int n, size_t bsz, double* dst, hipStream_t st) {
  const size_t total = (size_t)n * bsz;
  const int grid = (int)((total + 255) / 256 < 8192 ? (total + 255) / 256 : 8192);
  hipLaunchKernelGGL(k_scatter, dim3(grid > 0 ? grid : 1), dim3(256), 0, st, src, slots, n, bsz, dst);
  return hipGetLastError();
}

}  // namespace mrb
