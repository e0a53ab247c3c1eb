// Argument records of the predictor kernels (mlp.hip); internal to the library.
#pragma once
#include "internal.hpp"

namespace mrb {

struct MlpPoolArgs {
  Topo topo;
  const double* u;
  int nf;
  float* feat;        // [n][nf*64]
};

struct MlpArgs {
  const float* p;     // parameters
  int nin, n;
  const float* x;     // [n][nin] raw features
  const float* mean;  // [nf] normalisation
  const float* std;
  float* xn;          // [n][nin] normalised features (saved for the gradient)
  float* z1;          // [n][64]
  float* a1;
  float* z2;
  float* a2;
  float* logits;      // [n][3]
  const int8_t* y;    // [n] labels
  const float* classw;// [3]
  float inv_wsum;     // 1 / sum of the batch's label weights
  float* loss;        // [n] per-sample weighted loss
  float* dl;          // [n][3]
  float* dz1;         // [n][64]
  float* dz2;
  float* g;           // gradient, parameter layout
};

struct MlpAdamArgs {
  float* p;
  const float* g;
  float* m;
  float* v;
  int n;
  float lr, b1, b2, eps, bc1, bc2;
};

int mlp_param_count(int nin);
hipError_t launch_pool(int bs, int grid, const MlpPoolArgs& a, hipStream_t st);
hipError_t launch_mlp_forward(const MlpArgs& a, hipStream_t st);
hipError_t launch_mlp_backward(const MlpArgs& a, hipStream_t st);  // loss, deltas, parameter gradients
hipError_t launch_adam(const MlpAdamArgs& a, hipStream_t st);
hipError_t launch_pred(const float* logits, int n, int8_t* pred, float* pmax, hipStream_t st);

}  // namespace mrb
