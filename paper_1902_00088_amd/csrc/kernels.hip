// HIP kernels of the block-multiresolution sweep (gfx950).
//
// Every kernel works on one block per workgroup iteration (grid-stride over the
// block list, so a launch is independent of the block count and can be replayed
// from a graph).  A block's synchronised values over block + halo are built in
// LDS by "painting": each leaf whose closed region touches the block (coarser
// leaves first, then same-level leaves including the block itself, then finer
// leaves) writes its lattice points that fall inside the tile, so a point held by
// several leaves ends with the value of the finest one (finer blocks own the
// redundant nodes, Sec. 2.2 and Sec. 2.5).  Points that lie inside a coarser leaf
// but off its lattice are then predicted from the painted coarse-lattice points
// with the 4th-order central midpoint rule, tensor product x -> y -> z (the
// prediction operator of Sec. 2.3).  The stencil work is bandwidth bound and uses
// plain vector ALUs (no MFMA).
#include "internal.hpp"

#include <hip/hip_runtime.h>

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
// base + q*stride (n = 4) combined by P4; x first, then y, then z.
template <int DIM, typename T, typename AT>
__device__ __forceinline__ T tensor_p(const AT& at, const int* base, const int* stride, const int* n) {
  T vz[4] = {T(0), T(0), T(0), T(0)};
  const int nz = DIM > 2 ? n[2] : 1;
  for (int iz = 0; iz < nz; ++iz) {
    T vy[4] = {T(0), T(0), T(0), T(0)};
    for (int iy = 0; iy < n[1]; ++iy) {
      T vx[4] = {T(0), T(0), T(0), T(0)};
      for (int ix = 0; ix < n[0]; ++ix)
        vx[ix] = at(base[0] + ix * stride[0], base[1] + iy * stride[1], DIM > 2 ? base[2] + iz * stride[2] : 0);
      vy[iy] = n[0] == 4 ? P4(vx[0], vx[1], vx[2], vx[3]) : vx[0];
    }
    vz[iz] = n[1] == 4 ? P4(vy[0], vy[1], vy[2], vy[3]) : vy[0];
  }
  return nz == 4 ? P4(vz[0], vz[1], vz[2], vz[3]) : vz[0];
}

template <int DIM, int BS, int H>
struct TileGeo {
  static constexpr int TW = BS + 2 * H;
  static constexpr int TSZ = Pow<DIM, TW>::v;
  static constexpr int NP = Pow<DIM, BS>::v;
  __device__ static __forceinline__ int at(int x, int y, int z) {
    return (x + H) + TW * (y + H) + (DIM > 2 ? TW * TW * (z + H) : 0);
  }
};

// Stage value sources: y = u (+ alpha * k), optionally shifted by a per-field offset.
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

// Paint the tile [-H, BS-1+H]^DIM of block d; group by group with a barrier in
// between so that finer leaves overwrite coarser ones.  mask (if non-null)
// receives dl + 2 for every painted point.
template <int DIM, int BS, int H, int NF, typename TT, typename SRC>
__device__ void paint(TT* tile, uint8_t* mask, const BlockDesc& d, const NbEntry* nb, const SRC& src) {
  using G = TileGeo<DIM, BS, H>;
  constexpr int NP = G::NP;
  int e = d.nb_begin;
  const int ng[3] = {d.n_coarse, d.n_same, d.n_fine};
  for (int g = 0; g < 3; ++g) {
    for (int q = 0; q < ng[g]; ++q, ++e) {
      const NbEntry E = nb[e];
      const int dl = E.dl;
      const int ext = dl > 0 ? (BS - 1) / 2 : (dl == 0 ? BS - 1 : 2 * (BS - 1));
      const int step = dl < 0 ? 2 : 1;
      int lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
      bool empty = false;
      for (int a = 0; a < DIM; ++a) {
        int a0 = max(E.o[a], -H), a1 = min(E.o[a] + ext, BS - 1 + H);
        if (dl < 0 && ((a0 - E.o[a]) & 1)) ++a0;
        if (a1 < a0) empty = true;
        lo[a] = a0;
        cnt[a] = (a1 - a0) / step + 1;
      }
      if (empty) continue;
      const int total = cnt[0] * cnt[1] * (DIM > 2 ? cnt[2] : 1);
      const size_t sbase = (size_t)E.slot * NF * NP;
      for (int p = threadIdx.x; p < total; p += blockDim.x) {
        int t[3] = {0, 0, 0}, s[3] = {0, 0, 0};
        int rem = p;
        t[0] = lo[0] + (rem % cnt[0]) * step;
        rem /= cnt[0];
        t[1] = lo[1] + (DIM > 2 ? (rem % cnt[1]) : rem) * step;
        if (DIM > 2) t[2] = lo[2] + (rem / cnt[1]) * step;
        for (int a = 0; a < DIM; ++a) {
          const int l = t[a] - E.o[a];
          s[a] = dl > 0 ? 2 * l : (dl == 0 ? l : l / 2);
        }
        const int sidx = s[0] + BS * s[1] + (DIM > 2 ? BS * BS * s[2] : 0);
        const int tidx = G::at(t[0], t[1], t[2]);
#pragma unroll
        for (int f = 0; f < NF; ++f) tile[f * G::TSZ + tidx] = src(sbase + (size_t)f * NP + sidx, f);
        if (mask) mask[tidx] = (uint8_t)(dl + 2);
      }
    }
    __syncthreads();
  }
}

template <int DIM, int BS, int H>
__device__ void clear_mask(uint8_t* mask) {
  using G = TileGeo<DIM, BS, H>;
  for (int p = threadIdx.x; p < G::TSZ; p += blockDim.x) mask[p] = 0;
  __syncthreads();
}

// Predict every unpainted point of [-HW, BS-1+HW]^DIM from the even (coarse
// lattice) points around it.
template <int DIM, int BS, int H, int HW, int NF, typename TT>
__device__ void predict_missing(TT* tile, const uint8_t* mask) {
  using G = TileGeo<DIM, BS, H>;
  constexpr int W2 = BS + 2 * HW;
  constexpr int TOT = Pow<DIM, W2>::v;
  for (int p = threadIdx.x; p < TOT; p += blockDim.x) {
    int t[3] = {0, 0, 0};
    t[0] = p % W2 - HW;
    t[1] = (p / W2) % W2 - HW;
    if (DIM > 2) t[2] = p / (W2 * W2) - HW;
    const int tidx = G::at(t[0], t[1], t[2]);
    if (mask[tidx]) continue;
    int base[3], stride[3] = {2, 2, 2}, n[3] = {1, 1, 1};
    for (int a = 0; a < 3; ++a) base[a] = t[a];
    for (int a = 0; a < DIM; ++a)
      if (t[a] & 1) { base[a] = t[a] - 3; n[a] = 4; }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const TT* T = tile + f * G::TSZ;
      auto at = [&](int x, int y, int z) { return T[G::at(x, y, z)]; };
      tile[f * G::TSZ + tidx] = tensor_p<DIM, TT>(at, base, stride, n);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// right-hand sides on a synchronised tile (advection)
// ---------------------------------------------------------------------------
template <int DIM, int BS, int H, typename TT, int PHYS>
__device__ __forceinline__ TT rhs_adv(const TT* T, const BlockDesc& d, int i, int j, int k, TT r,
                                      const Physics& ph, double cfac, int nl, int shift) {
  using G = TileGeo<DIM, BS, H>;
  TT dx = D4(T[G::at(i - 2, j, k)], T[G::at(i - 1, j, k)], T[G::at(i + 1, j, k)], T[G::at(i + 2, j, k)], r);
  TT dy = D4(T[G::at(i, j - 2, k)], T[G::at(i, j - 1, k)], T[G::at(i, j + 1, k)], T[G::at(i, j + 2, k)], r);
  if constexpr (PHYS == 0) {
    TT c0, c1, c2;
    if constexpr (sizeof(TT) == 8) { c0 = ph.c[0]; c1 = ph.c[1]; c2 = ph.c[2]; }
    else { c0 = ph.cf[0]; c1 = ph.cf[1]; c2 = ph.cf[2]; }
    TT acc = c0 * dx;
    acc = acc + c1 * dy;
    if constexpr (DIM > 2) {
      TT dz = D4(T[G::at(i, j, k - 2)], T[G::at(i, j, k - 1)], T[G::at(i, j, k + 1)], T[G::at(i, j, k + 2)], r);
      acc = acc + c2 * dz;
    }
    return -acc;
  } else {
    int gx = d.c[0] * (BS - 1) + i;
    int gy = d.c[1] * (BS - 1) + j;
    if (gx >= nl) gx -= nl;
    if (gy >= nl) gy -= nl;
    gx <<= shift;
    gy <<= shift;
    const double U = (ph.s2[gx] * ph.s[gy]) * cfac;
    const double W = -((ph.s2[gy] * ph.s[gx]) * cfac);
    return -(((TT)U * dx) + ((TT)W * dy));
  }
}

// ---------------------------------------------------------------------------
// fused stage kernel: paint y_s, predict missing ghosts, RHS, store
// ---------------------------------------------------------------------------
template <int DIM, int BS, int HW, int NF, typename TT, typename KT, int PHYS>
__global__ void __launch_bounds__(kNT) k_stage(StageArgs A) {
  constexpr int H = HW + 2;
  using G = TileGeo<DIM, BS, H>;
  constexpr int NP = G::NP;
  extern __shared__ __align__(16) char smem[];
  TT* tile = reinterpret_cast<TT*>(smem);
  uint8_t* mask = reinterpret_cast<uint8_t*>(smem + sizeof(TT) * NF * G::TSZ);
  const int nblk = A.list ? A.list_n : *A.count;
  for (int bi = blockIdx.x; bi < nblk; bi += gridDim.x) {
    const int b = A.list ? A.list[bi] : bi;
    const BlockDesc d = A.blk[b];
    clear_mask<DIM, BS, H>(mask);
    if (A.stage == 1) {
      YSrc<TT, KT, false> src{A.u, nullptr, 0.0, A.off};
      paint<DIM, BS, H, NF, TT>(tile, mask, d, A.nb, src);
    } else {
      YSrc<TT, KT, true> src{A.u, (const KT*)A.kprev, A.alpha, A.off};
      paint<DIM, BS, H, NF, TT>(tile, mask, d, A.nb, src);
    }
    predict_missing<DIM, BS, H, HW, NF, TT>(tile, mask);
    TT r;
    if constexpr (sizeof(TT) == 8) r = A.lt.r[d.level];
    else r = A.lt.rf[d.level];
    const int nl = A.lt.nl[d.level];
    const int shift = A.ph.jmax - d.level;
    const size_t base = (size_t)d.slot * NF * NP;
    for (int p = threadIdx.x; p < NP; p += blockDim.x) {
      const int i = p % BS, j = (p / BS) % BS, k = DIM > 2 ? p / (BS * BS) : 0;
      const TT kv = rhs_adv<DIM, BS, H, TT, PHYS>(tile, d, i, j, k, r, A.ph, A.cfac, nl, shift);
      if (A.stage < 4) {
        ((KT*)A.kout)[base + p] = (KT)kv;
      } else {
        const double k1 = (double)((const KT*)A.k1)[base + p];
        const double k2 = (double)((const KT*)A.k2)[base + p];
        const double k3 = (double)((const KT*)A.k3)[base + p];
        const double k4 = (double)kv;
        A.unew[base + p] = A.u[base + p] + A.h6 * ((k1 + k4) + 2.0 * (k2 + k3));
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// plain form: ghost fill into HBM, then a separate RHS + update kernel
// ---------------------------------------------------------------------------
template <int DIM, int BS, int HW, int NF>
__global__ void __launch_bounds__(kNT) k_ghost(StageArgs A) {
  constexpr int H = HW + 2;
  using G = TileGeo<DIM, BS, H>;
  constexpr int GW = BS + 2 * HW;
  constexpr int GSZ = Pow<DIM, GW>::v;
  extern __shared__ __align__(16) char smem[];
  double* tile = reinterpret_cast<double*>(smem);
  uint8_t* mask = reinterpret_cast<uint8_t*>(smem + sizeof(double) * NF * G::TSZ);
  const int nblk = A.list ? A.list_n : *A.count;
  for (int bi = blockIdx.x; bi < nblk; bi += gridDim.x) {
    const int b = A.list ? A.list[bi] : bi;
    const BlockDesc d = A.blk[b];
    clear_mask<DIM, BS, H>(mask);
    if (A.stage == 1) {
      YSrc<double, double, false> src{A.u, nullptr, 0.0, A.off};
      paint<DIM, BS, H, NF, double>(tile, mask, d, A.nb, src);
    } else {
      YSrc<double, double, true> src{A.u, (const double*)A.kprev, A.alpha, A.off};
      paint<DIM, BS, H, NF, double>(tile, mask, d, A.nb, src);
    }
    predict_missing<DIM, BS, H, HW, NF, double>(tile, mask);
    double* g = A.ghost + (size_t)d.slot * NF * GSZ;
    for (int p = threadIdx.x; p < GSZ; p += blockDim.x) {
      const int x = p % GW - HW, y = (p / GW) % GW - HW, z = DIM > 2 ? p / (GW * GW) - HW : 0;
#pragma unroll
      for (int f = 0; f < NF; ++f) g[(size_t)f * GSZ + p] = tile[f * G::TSZ + G::at(x, y, z)];
    }
    __syncthreads();
  }
}

template <int DIM, int BS, int HW, int NF, int PHYS>
__global__ void __launch_bounds__(kNT) k_rhs_plain(StageArgs A) {
  using G = TileGeo<DIM, BS, HW>;
  constexpr int NP = G::NP;
  const int nblk = A.list ? A.list_n : *A.count;
  for (int bi = blockIdx.x; bi < nblk; bi += gridDim.x) {
    const int b = A.list ? A.list[bi] : bi;
    const BlockDesc d = A.blk[b];
    const double* T = A.ghost + (size_t)d.slot * NF * G::TSZ;
    const double r = A.lt.r[d.level];
    const int nl = A.lt.nl[d.level];
    const int shift = A.ph.jmax - d.level;
    const size_t base = (size_t)d.slot * NF * NP;
    for (int p = threadIdx.x; p < NP; p += blockDim.x) {
      const int i = p % BS, j = (p / BS) % BS, k = DIM > 2 ? p / (BS * BS) : 0;
      const double kv = rhs_adv<DIM, BS, HW, double, PHYS>(T, d, i, j, k, r, A.ph, A.cfac, nl, shift);
      if (A.stage < 4) {
        ((double*)A.kout)[base + p] = kv;
      } else {
        const double k1 = ((const double*)A.k1)[base + p];
        const double k2 = ((const double*)A.k2)[base + p];
        const double k3 = ((const double*)A.k3)[base + p];
        A.unew[base + p] = A.u[base + p] + A.h6 * ((k1 + kv) + 2.0 * (k2 + k3));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// multiresolution analysis: details d = u - P(R(u)), per-field max, flag;
// redundant nodes owned by finer neighbours are written back to the pool
// ---------------------------------------------------------------------------
__device__ __forceinline__ double nanmax(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}

template <int DIM, int BS, int NF>
__global__ void __launch_bounds__(kNT) k_mr(MrArgs A) {
  constexpr int H = 2;
  using G = TileGeo<DIM, BS, H>;
  constexpr int NP = G::NP;
  extern __shared__ __align__(16) char smem[];
  double* tile = reinterpret_cast<double*>(smem);
  uint8_t* mask = reinterpret_cast<uint8_t*>(smem + sizeof(double) * NF * G::TSZ);
  __shared__ double red[kNT / 64][4];
  const int nblk = *A.count;
  for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
    const BlockDesc d = A.blk[b];
    clear_mask<DIM, BS, H>(mask);
    YSrc<double, double, false> src{A.u, nullptr, 0.0, nullptr};
    paint<DIM, BS, H, NF, double>(tile, mask, d, A.nb, src);
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    const size_t base = (size_t)d.slot * NF * NP;
    for (int p = threadIdx.x; p < NP; p += blockDim.x) {
      int ii[3] = {p % BS, (p / BS) % BS, DIM > 2 ? p / (BS * BS) : 0};
      const int tidx = G::at(ii[0], ii[1], ii[2]);
      bool bnd = false, allEven = true;
      for (int a = 0; a < DIM; ++a) {
        if (ii[a] == 0 || ii[a] == BS - 1) bnd = true;
        if (ii[a] & 1) allEven = false;
      }
      if (bnd && mask[tidx] == 3) {
#pragma unroll
        for (int f = 0; f < NF; ++f) A.u[base + (size_t)f * NP + p] = tile[f * G::TSZ + tidx];
      }
      if (allEven) continue;   // restriction then prediction returns these nodes unchanged
      int bb[3], stride[3] = {2, 2, 2}, n[3] = {1, 1, 1};
      for (int a = 0; a < 3; ++a) bb[a] = ii[a];
      for (int a = 0; a < DIM; ++a)
        if (ii[a] & 1) { bb[a] = ii[a] - 3; n[a] = 4; }
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double* T = tile + f * G::TSZ;
        auto at = [&](int x, int y, int z) { return T[G::at(x, y, z)]; };
        const double pred = tensor_p<DIM, double>(at, bb, stride, n);
        const double dd = fabs(T[tidx] - pred);
        m[f] = nanmax(m[f], dd);
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      double v = m[f];
      for (int off = 32; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off, 64));
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][f] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      bool coarse = d.level > 1;
      for (int f = 0; f < NF; ++f) {
        double v = red[0][f];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = nanmax(v, red[w][f]);
        A.maxd[(size_t)b * NF + f] = v;
        if (!(v < A.thr[f])) coarse = false;
      }
      A.flags[b] = coarse ? (int8_t)-1 : (int8_t)0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// refinement: children take the synchronised value at level l+1 -- the finer
// neighbour's stored value where one holds the node, else the parent tile value
// (even nodes) or its prediction (odd nodes)
// ---------------------------------------------------------------------------
template <int DIM, int BS, int NF>
__global__ void __launch_bounds__(kNT) k_refine(RefineArgs A) {
  constexpr int HW = 2, H = 4;
  using G = TileGeo<DIM, BS, H>;
  constexpr int NP = G::NP;
  constexpr int NCH = 1 << DIM;
  extern __shared__ __align__(16) char smem[];
  double* tile = reinterpret_cast<double*>(smem);
  uint8_t* mask = reinterpret_cast<uint8_t*>(smem + sizeof(double) * NF * G::TSZ);
  const int nref = *A.count;
  for (int r = blockIdx.x; r < nref; r += gridDim.x) {
    const RefineDesc R = A.ref[r];
    const BlockDesc d = A.blk[R.blk];
    clear_mask<DIM, BS, H>(mask);
    YSrc<double, double, false> src{A.u, nullptr, 0.0, nullptr};
    paint<DIM, BS, H, NF, double>(tile, mask, d, A.nb, src);
    predict_missing<DIM, BS, H, HW, NF, double>(tile, mask);
    const int fine0 = d.nb_begin + d.n_coarse + d.n_same;
    for (int p = threadIdx.x; p < NCH * NP; p += blockDim.x) {
      const int ch = p / NP, q = p % NP;
      int Q[3] = {q % BS, (q / BS) % BS, DIM > 2 ? q / (BS * BS) : 0};
      bool bnd = false, allEven = true;
      for (int a = 0; a < DIM; ++a) {
        Q[a] += ((ch >> a) & 1) * (BS - 1);
        if (Q[a] == 0 || Q[a] == 2 * (BS - 1)) bnd = true;
        if (Q[a] & 1) allEven = false;
      }
      const size_t cbase = (size_t)R.child[ch] * NF * NP + q;
      int src_slot = -1, sidx = 0;
      if (bnd && !allEven) {
        for (int e = fine0; e < fine0 + d.n_fine; ++e) {
          const NbEntry E = A.nb[e];
          bool in = true;
          int s = 0, mul = 1;
          for (int a = 0; a < DIM; ++a) {
            const int l = Q[a] - 2 * E.o[a];
            if (l < 0 || l > BS - 1) in = false;
            s += l * mul;
            mul *= BS;
          }
          if (in) { src_slot = E.slot; sidx = s; break; }
        }
      }
      if (src_slot >= 0) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
          A.u[cbase + (size_t)f * NP] = A.u[((size_t)src_slot * NF + f) * NP + sidx];
        continue;
      }
      int bb[3] = {0, 0, 0}, stride[3] = {1, 1, 1}, n[3] = {1, 1, 1};
      for (int a = 0; a < DIM; ++a) {
        if (Q[a] & 1) { bb[a] = (Q[a] - 3) / 2; n[a] = 4; }
        else bb[a] = Q[a] / 2;
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double* T = tile + f * G::TSZ;
        auto at = [&](int x, int y, int z) { return T[G::at(x, y, z)]; };
        A.u[cbase + (size_t)f * NP] = tensor_p<DIM, double>(at, bb, stride, n);
      }
    }
    __syncthreads();
  }
}

// coarsening: the mother keeps every second node of her children (restriction R);
// a node shared by several children is taken from the lowest child index
template <int DIM, int BS, int NF>
__global__ void __launch_bounds__(kNT) k_coarsen(CoarsenArgs A) {
  constexpr int NP = Pow<DIM, BS>::v;
  const int nfam = *A.count;
  const long total = (long)nfam * NP;
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < total; p += (long)gridDim.x * blockDim.x) {
    const int fi = (int)(p / NP), q = (int)(p % NP);
    const FamilyDesc F = A.fam[fi];
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

// read-back of synchronised block values in forest order
template <int DIM, int BS, int NF>
__global__ void __launch_bounds__(kNT) k_read(ReadArgs A) {
  constexpr int H = 0;
  using G = TileGeo<DIM, BS, H>;
  constexpr int NP = G::NP;
  extern __shared__ __align__(16) char smem[];
  double* tile = reinterpret_cast<double*>(smem);
  const int nblk = *A.count;
  for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
    const BlockDesc d = A.blk[b];
    YSrc<double, double, false> src{A.u, nullptr, 0.0, nullptr};
    paint<DIM, BS, H, NF, double>(tile, nullptr, d, A.nb, src);
    for (int p = threadIdx.x; p < NF * NP; p += blockDim.x) A.out[(size_t)b * NF * NP + p] = tile[p];
    __syncthreads();
  }
}

// whole-block copy from a contiguous [n][bsz] array into pool slots
__global__ void __launch_bounds__(kNT) k_scatter(const double* src, const int* slots, int n, size_t bsz, double* dst) {
  const size_t total = (size_t)n * bsz;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < total; p += (size_t)gridDim.x * blockDim.x) {
    const size_t b = p / bsz, q = p % bsz;
    dst[(size_t)slots[b] * bsz + q] = src[p];
  }
}

hipError_t launch_scatter(const double* src, const int* slots, int n, size_t bsz, double* dst, hipStream_t st) {
  const size_t total = (size_t)n * bsz;
  const int grid = (int)std::min<size_t>(8192, (total + kNT - 1) / kNT);
  hipLaunchKernelGGL(k_scatter, dim3(grid > 0 ? grid : 1), dim3(kNT), 0, st, src, slots, n, bsz, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename K>
static hipError_t prep(K kern, size_t lds) {
  if (lds > 65536) return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

template <int DIM, int BS, int HW, int NF>
static hipError_t stage_impl(int precision, int grid, const StageArgs& a, hipStream_t st) {
  constexpr int H = HW + 2;
  using G = TileGeo<DIM, BS, H>;
  const bool swirl = a.ph.kind == 1;
  if (precision == 0) {
    const size_t lds = sizeof(double) * NF * G::TSZ + G::TSZ;
    auto kern = swirl ? k_stage<DIM, BS, HW, NF, double, double, 1> : k_stage<DIM, BS, HW, NF, double, double, 0>;
    hipError_t e = prep(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kNT), lds, st, a);
  } else {
    const size_t lds = sizeof(float) * NF * G::TSZ + G::TSZ;
    auto kern = swirl ? k_stage<DIM, BS, HW, NF, float, float, 1> : k_stage<DIM, BS, HW, NF, float, float, 0>;
    hipError_t e = prep(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kNT), lds, st, a);
  }
  return hipGetLastError();
}

template <int DIM, int BS, int HW, int NF>
static hipError_t ghost_impl(int grid, const StageArgs& a, hipStream_t st) {
  constexpr int H = HW + 2;
  using G = TileGeo<DIM, BS, H>;
  const size_t lds = sizeof(double) * NF * G::TSZ + G::TSZ;
  auto kern = k_ghost<DIM, BS, HW, NF>;
  hipError_t e = prep(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kNT), lds, st, a);
  return hipGetLastError();
}

template <int DIM, int BS, int HW, int NF>
static hipError_t rhs_plain_impl(int grid, const StageArgs& a, hipStream_t st) {
  if (a.ph.kind == 1) hipLaunchKernelGGL((k_rhs_plain<DIM, BS, HW, NF, 1>), dim3(grid), dim3(kNT), 0, st, a);
  else hipLaunchKernelGGL((k_rhs_plain<DIM, BS, HW, NF, 0>), dim3(grid), dim3(kNT), 0, st, a);
  return hipGetLastError();
}

template <int DIM, int BS, int NF>
static hipError_t mr_impl(int grid, const MrArgs& a, hipStream_t st) {
  using G = TileGeo<DIM, BS, 2>;
  const size_t lds = sizeof(double) * NF * G::TSZ + G::TSZ;
  auto kern = k_mr<DIM, BS, NF>;
  hipError_t e = prep(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kNT), lds, st, a);
  return hipGetLastError();
}

template <int DIM, int BS, int NF>
static hipError_t refine_impl(int grid, const RefineArgs& a, hipStream_t st) {
  using G = TileGeo<DIM, BS, 4>;
  const size_t lds = sizeof(double) * NF * G::TSZ + G::TSZ;
  auto kern = k_refine<DIM, BS, NF>;
  hipError_t e = prep(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kNT), lds, st, a);
  return hipGetLastError();
}

template <int DIM, int BS, int NF>
static hipError_t read_impl(int grid, const ReadArgs& a, hipStream_t st) {
  using G = TileGeo<DIM, BS, 0>;
  const size_t lds = sizeof(double) * NF * G::TSZ;
  auto kern = k_read<DIM, BS, NF>;
  hipError_t e = prep(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kNT), lds, st, a);
  return hipGetLastError();
}

#define MRB_SHAPES(X) \
  X(2, 17, 2, 1)      \
  X(2, 33, 2, 1)      \
  X(3, 17, 2, 1)

bool shape_supported(const Shape& s) {
#define X(D, B, W, F) if (s.dim == D && s.bs == B && s.hw == W && s.nf == F) return true;
  MRB_SHAPES(X)
#undef X
  return false;
}

hipError_t launch_stage(const Shape& s, int precision, int plain_rhs, int grid, const StageArgs& a, hipStream_t st) {
#define X(D, B, W, F)                                                        \
  if (s.dim == D && s.bs == B && s.hw == W && s.nf == F)                     \
    return plain_rhs ? rhs_plain_impl<D, B, W, F>(grid, a, st) : stage_impl<D, B, W, F>(precision, grid, a, st);
  MRB_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_ghost(const Shape& s, int grid, const StageArgs& a, hipStream_t st) {
#define X(D, B, W, F) if (s.dim == D && s.bs == B && s.hw == W && s.nf == F) return ghost_impl<D, B, W, F>(grid, a, st);
  MRB_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_mr(const Shape& s, int grid, const MrArgs& a, hipStream_t st) {
#define X(D, B, W, F) if (s.dim == D && s.bs == B && s.hw == W && s.nf == F) return mr_impl<D, B, F>(grid, a, st);
  MRB_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_refine(const Shape& s, int grid, const RefineArgs& a, hipStream_t st) {
#define X(D, B, W, F) if (s.dim == D && s.bs == B && s.hw == W && s.nf == F) return refine_impl<D, B, F>(grid, a, st);
  MRB_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_coarsen(const Shape& s, int grid, const CoarsenArgs& a, hipStream_t st) {
#define X(D, B, W, F)                                                                   \
  if (s.dim == D && s.bs == B && s.hw == W && s.nf == F) {                              \
    hipLaunchKernelGGL((k_coarsen<D, B, F>), dim3(grid), dim3(kNT), 0, st, a);          \
    return hipGetLastError();                                                           \
  }
  MRB_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_read(const Shape& s, int grid, const ReadArgs& a, hipStream_t st) {
#define X(D, B, W, F) if (s.dim == D && s.bs == B && s.hw == W && s.nf == F) return read_impl<D, B, F>(grid, a, st);
  MRB_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace mrb
