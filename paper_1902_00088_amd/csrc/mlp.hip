// Learned refinement predictor on the GPU: block features (8 x 8 average pool of
// every field of the synchronised block), a nin -> 64 -> 64 -> 3 MLP with GELU,
// class-weighted softmax cross-entropy, backward pass and Adam.  FP32 arithmetic;
// the per-parameter gradient reduction over the batch accumulates in FP64 in a
// fixed order (deterministic, no atomics).  The layers are tiny (a batch of 1024
// is ~20 MFLOP), so plain FMA loops with weights read through the caches do; the
// parameter vector layout is W1[nin][64], b1[64], W2[64][64], b2[64], W3[64][3], b3[3].
#include "internal.hpp"
#include "mlp.hpp"

#include <hip/hip_runtime.h>

namespace mrb {

namespace {

constexpr int HID = 64, NOUT = 3;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

struct Off {
  int w1, b1, w2, b2, w3, b3, n;
  __device__ __host__ explicit Off(int nin) {
    w1 = 0;
    b1 = nin * HID;
    w2 = b1 + HID;
    b2 = w2 + HID * HID;
    w3 = b2 + HID;
    b3 = w3 + HID * NOUT;
    n = b3 + NOUT;
  }
};

// features of every block: gather the synchronised block (no halo) and average each
// field over 8 x 8 bins of w = (bs-1)/8 nodes (y outer, x inner, FP64)
template <int BS>
__global__ void __launch_bounds__(256) k_pool(MlpPoolArgs A) {
  constexpr int NPT = BS * BS;
  constexpr int W = (BS - 1) / 8;
  extern __shared__ __align__(16) char smem[];
  double* tile = reinterpret_cast<double*>(smem);
  const int nblk = A.topo.h.n_blocks;
  for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
    const BlockDesc d = A.topo.blk()[b];
    // owner of each node: the block itself except on its boundary, where a finer
    // neighbour may hold the node; a same-level neighbour holds equal values
    for (int p = threadIdx.x; p < A.nf * NPT; p += blockDim.x) {
      const int f = p / NPT, q = p % NPT, x = q % BS, y = q / BS;
      double v = A.u[((size_t)d.slot * A.nf + f) * NPT + q];
      if (x == 0 || y == 0 || x == BS - 1 || y == BS - 1) {
        for (int e = 0; e < d.n_ent; ++e) {
          const NbEntry E = A.topo.nb(b)[e];
          if (E.dl <= 0) continue;
          const int lx = x - E.o[0], ly = y - E.o[1];
          if (lx >= 0 && lx <= (BS - 1) / 2 && ly >= 0 && ly <= (BS - 1) / 2) {
            v = A.u[((size_t)E.slot * A.nf + f) * NPT + 2 * lx + BS * 2 * ly];
            break;
          }
        }
      }
      tile[p] = v;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < A.nf * 64; p += blockDim.x) {
      const int f = p / 64, bin = p % 64, bx = bin % 8, by = bin / 8;
      double s = 0.0;
      for (int y = by * W; y < by * W + W; ++y)
        for (int x = bx * W; x < bx * W + W; ++x) s = s + tile[f * NPT + y * BS + x];
      A.feat[(size_t)b * A.nf * 64 + p] = (float)(s / (double)(W * W));
    }
    __syncthreads();
  }
}

// forward pass, one wave per sample: normalise, two GELU layers, logits
__global__ void __launch_bounds__(64) k_fwd(MlpArgs A) {
  __shared__ float xs[256], a1[HID], a2[HID];
  const Off o(A.nin);
  const int j = threadIdx.x;
  for (int b = blockIdx.x; b < A.n; b += gridDim.x) {
    for (int k = j; k < A.nin; k += 64) {
      const int f = k / 64;
      const float xn = (A.x[(size_t)b * A.nin + k] - A.mean[f]) / A.std[f];
      xs[k] = xn;
      if (A.xn) A.xn[(size_t)b * A.nin + k] = xn;
    }
    __syncthreads();
    float z = A.p[o.b1 + j];
    for (int k = 0; k < A.nin; ++k) z = z + xs[k] * A.p[o.w1 + k * HID + j];
    if (A.z1) A.z1[(size_t)b * HID + j] = z;
    a1[j] = gelu(z);
    __syncthreads();
    z = A.p[o.b2 + j];
    for (int k = 0; k < HID; ++k) z = z + a1[k] * A.p[o.w2 + k * HID + j];
    if (A.z2) A.z2[(size_t)b * HID + j] = z;
    const float g2 = gelu(z);
    a2[j] = g2;
    if (A.a1) A.a1[(size_t)b * HID + j] = a1[j];
    if (A.a2) A.a2[(size_t)b * HID + j] = g2;
    __syncthreads();
    if (j < NOUT) {
      float l = A.p[o.b3 + j];
      for (int k = 0; k < HID; ++k) l = l + a2[k] * A.p[o.w3 + k * NOUT + j];
      A.logits[(size_t)b * NOUT + j] = l;
    }
    __syncthreads();
  }
}

// weighted softmax cross-entropy: per-sample loss and dL/dlogits
__global__ void __launch_bounds__(256) k_ce(MlpArgs A) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < A.n; b += gridDim.x * blockDim.x) {
    const float* l = A.logits + (size_t)b * NOUT;
    const float m = fmaxf(l[0], fmaxf(l[1], l[2]));
    const float e0 = expf(l[0] - m), e1 = expf(l[1] - m), e2 = expf(l[2] - m);
    const float s = e0 + e1 + e2;
    const float pr[3] = {e0 / s, e1 / s, e2 / s};
    const int y = A.y[b];
    const float w = A.classw[y];
    A.loss[b] = -logf(pr[y]) * w * A.inv_wsum;
    for (int c = 0; c < NOUT; ++c) A.dl[(size_t)b * NOUT + c] = (pr[c] - (c == y ? 1.0f : 0.0f)) * (w * A.inv_wsum);
  }
}

// backward deltas, one wave per sample
__global__ void __launch_bounds__(64) k_bwd(MlpArgs A) {
  __shared__ float dz2[HID];
  const Off o(A.nin);
  const int j = threadIdx.x;
  for (int b = blockIdx.x; b < A.n; b += gridDim.x) {
    const float* dl = A.dl + (size_t)b * NOUT;
    float da2 = 0.0f;
    for (int c = 0; c < NOUT; ++c) da2 = da2 + dl[c] * A.p[o.w3 + j * NOUT + c];
    const float d2 = da2 * gelu_grad(A.z2[(size_t)b * HID + j]);
    dz2[j] = d2;
    A.dz2[(size_t)b * HID + j] = d2;
    __syncthreads();
    float da1 = 0.0f;
    for (int k = 0; k < HID; ++k) da1 = da1 + dz2[k] * A.p[o.w2 + j * HID + k];
    A.dz1[(size_t)b * HID + j] = da1 * gelu_grad(A.z1[(size_t)b * HID + j]);
    __syncthreads();
  }
}

// parameter gradients: one thread per parameter, sum over the batch in order (FP64)
__global__ void __launch_bounds__(256) k_wgrad(MlpArgs A) {
  const Off o(A.nin);
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < o.n; q += gridDim.x * blockDim.x) {
    double s = 0.0;
    if (q < o.b1) {
      const int k = q / HID, j = q % HID;
      for (int b = 0; b < A.n; ++b) s += (double)A.xn[(size_t)b * A.nin + k] * (double)A.dz1[(size_t)b * HID + j];
    } else if (q < o.w2) {
      const int j = q - o.b1;
      for (int b = 0; b < A.n; ++b) s += (double)A.dz1[(size_t)b * HID + j];
    } else if (q < o.b2) {
      const int k = (q - o.w2) / HID, j = (q - o.w2) % HID;
      for (int b = 0; b < A.n; ++b) s += (double)A.a1[(size_t)b * HID + k] * (double)A.dz2[(size_t)b * HID + j];
    } else if (q < o.w3) {
      const int j = q - o.b2;
      for (int b = 0; b < A.n; ++b) s += (double)A.dz2[(size_t)b * HID + j];
    } else if (q < o.b3) {
      const int k = (q - o.w3) / NOUT, c = (q - o.w3) % NOUT;
      for (int b = 0; b < A.n; ++b) s += (double)A.a2[(size_t)b * HID + k] * (double)A.dl[(size_t)b * NOUT + c];
    } else {
      const int c = q - o.b3;
      for (int b = 0; b < A.n; ++b) s += (double)A.dl[(size_t)b * NOUT + c];
    }
    A.g[q] = (float)s;
  }
}

__global__ void __launch_bounds__(256) k_adam(MlpAdamArgs A) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < A.n; q += gridDim.x * blockDim.x) {
    const float g = A.g[q];
    const float m = A.b1 * A.m[q] + (1.0f - A.b1) * g;
    const float v = A.b2 * A.v[q] + (1.0f - A.b2) * g * g;
    A.m[q] = m;
    A.v[q] = v;
    A.p[q] = A.p[q] - A.lr * (m / A.bc1) / (sqrtf(v / A.bc2) + A.eps);
  }
}

// prediction from logits: argmax class and its softmax probability
__global__ void __launch_bounds__(256) k_pred(const float* logits, int n, int8_t* pred, float* pmax) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < n; b += gridDim.x * blockDim.x) {
    const float* l = logits + (size_t)b * NOUT;
    int c = 0;
    if (l[1] > l[c]) c = 1;
    if (l[2] > l[c]) c = 2;
    const float s = expf(l[0] - l[c]) + expf(l[1] - l[c]) + expf(l[2] - l[c]);
    pred[b] = (int8_t)c;
    pmax[b] = 1.0f / s;
  }
}

}  // namespace

int mlp_param_count(int nin) { return Off(nin).n; }

hipError_t launch_pred(const float* logits, int n, int8_t* pred, float* pmax, hipStream_t st) {
  const int g = (n + 255) / 256;
  hipLaunchKernelGGL(k_pred, dim3(g > 0 ? g : 1), dim3(256), 0, st, logits, n, pred, pmax);
  return hipGetLastError();
}

hipError_t launch_pool(int bs, int grid, const MlpPoolArgs& a, hipStream_t st) {
  const size_t lds = sizeof(double) * a.nf * bs * bs;
  if (bs == 33) hipLaunchKernelGGL(k_pool<33>, dim3(grid), dim3(256), lds, st, a);
  else if (bs == 17) hipLaunchKernelGGL(k_pool<17>, dim3(grid), dim3(256), lds, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpArgs& a, hipStream_t st) {
  const int grid = a.n < 4096 ? (a.n > 0 ? a.n : 1) : 4096;
  hipLaunchKernelGGL(k_fwd, dim3(grid), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const MlpArgs& a, hipStream_t st) {
  const int g1 = (a.n + 255) / 256;
  hipLaunchKernelGGL(k_ce, dim3(g1 > 0 ? g1 : 1), dim3(256), 0, st, a);
  const int grid = a.n < 4096 ? (a.n > 0 ? a.n : 1) : 4096;
  hipLaunchKernelGGL(k_bwd, dim3(grid), dim3(64), 0, st, a);
  const int np = Off(a.nin).n;
  hipLaunchKernelGGL(k_wgrad, dim3((np + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_adam(const MlpAdamArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace mrb
