// Learned neighbor proposal: the embedding network and its training kernels.
//
// The correlation metric of the Gneiting class has no exact Euclidean embedding
// (Sec. "Correlation-based Vecchia neighbor selection"), which is why the paper
// searches it with a cover tree. Here a small MLP maps each point (standardised
// coordinates and time, plus the five log hyperparameters that shape the
// correlation) to a 16-d embedding whose Euclidean distances propose candidates;
// the exact correlation key then reranks them (neighbors.hip).
//
// Network: 8 -> 64 -> 64 -> 64 -> 16, ReLU on the hidden layers, FP32
// parameters packed as W1[8][64], b1[64], W2[64][64], b2[64], W3[64][64],
// b3[64], W4[64][16], b4[16] (row-major, h_out = h_in W + b).
//
// gfx950 design: the layers are tiny (9936 parameters, 40 KB) and stay in LDS;
// the forward pass runs one row per thread with LDS-broadcast weights. The
// backward pass works on blocks of 64 rows: back-propagated activations go
// through LDS, each block writes its partial parameter gradient, and a second
// kernel sums the partials in FP64 in block order (deterministic).
#include "internal.hpp"

namespace vif {

namespace {

constexpr int NI = 8, NH = 64, NO = 16;
constexpr int OW1 = 0, OB1 = OW1 + NI * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH,
              OW3 = OB2 + NH, OB3 = OW3 + NH * NH, OW4 = OB3 + NH, OB4 = OW4 + NH * NO,
              NPAR = OB4 + NO;
static_assert(NPAR == 9936, "parameter count");

__device__ __forceinline__ void load_params(float* sp, const float* __restrict__ params) {
  for (int e = threadIdx.x; e < NPAR; e += blockDim.x) sp[e] = params[e];
}

// ---------------------------------------------------------------- features ----
__global__ void features_kernel(int64_t n, const double* __restrict__ sx,
                                const double* __restrict__ sy, const double* __restrict__ t,
                                FeatArgs F, float* __restrict__ X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float* x = X + i * NI;
  x[0] = (float)((sx[i] - F.cx) / F.ss);
  x[1] = (float)((sy[i] - F.cy) / F.ss);
  x[2] = (float)((t[i] - F.ct) / F.st);
#pragma unroll
  for (int c = 0; c < 5; ++c) x[3 + c] = (float)F.hyper[c];
}

// ----------------------------------------------------------------- forward ----
__global__ __launch_bounds__(256) void mlp_forward_kernel(int64_t rows,
                                                          const float* __restrict__ params,
                                                          const float* __restrict__ X,
                                                          float* __restrict__ E,
                                                          float* __restrict__ H) {
  __shared__ float sp[NPAR];
  load_params(sp, params);
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  float x[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) x[i] = X[r * NI + i];
  float a[NH], b[NH];
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    float s = sp[OB1 + j];
#pragma unroll
    for (int i = 0; i < NI; ++i) s += x[i] * sp[OW1 + i * NH + j];
    a[j] = fmaxf(s, 0.f);
  }
  if (H) {
#pragma unroll
    for (int j = 0; j < NH; ++j) H[(r * 3 + 0) * NH + j] = a[j];
  }
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    float s = sp[OB2 + j];
#pragma unroll
    for (int i = 0; i < NH; ++i) s += a[i] * sp[OW2 + i * NH + j];
    b[j] = fmaxf(s, 0.f);
  }
  if (H) {
#pragma unroll
    for (int j = 0; j < NH; ++j) H[(r * 3 + 1) * NH + j] = b[j];
  }
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    float s = sp[OB3 + j];
#pragma unroll
    for (int i = 0; i < NH; ++i) s += b[i] * sp[OW3 + i * NH + j];
    a[j] = fmaxf(s, 0.f);
  }
  if (H) {
#pragma unroll
    for (int j = 0; j < NH; ++j) H[(r * 3 + 2) * NH + j] = a[j];
  }
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    float s = sp[OB4 + j];
#pragma unroll
    for (int i = 0; i < NH; ++i) s += a[i] * sp[OW4 + i * NO + j];
    E[r * NO + j] = s;
  }
}

// ---------------------------------------------------------------- backward ----
constexpr int BR = 64;  // rows per block

// Partial gradient of sum(dE * E) over rows [64 blk, 64 blk + 64) into part[blk].
__global__ __launch_bounds__(256) void mlp_backward_kernel(int64_t rows,
                                                           const float* __restrict__ params,
                                                           const float* __restrict__ X,
                                                           const float* __restrict__ H,
                                                           const float* __restrict__ dE,
                                                           float* __restrict__ part) {
  __shared__ float sx[BR][NI];
  __shared__ float sh[3][BR][NH + 1];  // h1, h2, h3 (post-ReLU)
  __shared__ float sg[3][BR][NH + 1];  // gradients at the pre-activations of layers 1..3
  __shared__ float se[BR][NO];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * BR;
  for (int e = tid; e < BR * NI; e += 256) {
    const int r = e / NI, c = e % NI;
    sx[r][c] = r0 + r < rows ? X[(r0 + r) * NI + c] : 0.f;
  }
  for (int e = tid; e < 3 * BR * NH; e += 256) {
    const int l = e / (BR * NH), rem = e % (BR * NH), r = rem / NH, c = rem % NH;
    sh[l][r][c] = r0 + r < rows ? H[((r0 + r) * 3 + l) * NH + c] : 0.f;
  }
  for (int e = tid; e < BR * NO; e += 256) {
    const int r = e / NO, c = e % NO;
    se[r][c] = r0 + r < rows ? dE[(r0 + r) * NO + c] : 0.f;
  }
  __syncthreads();
  // layer 3: g3 = (dE W4^T) * (h3 > 0)
  for (int e = tid; e < BR * NH; e += 256) {
    const int r = e / NH, j = e % NH;
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < NO; ++k) s += se[r][k] * params[OW4 + j * NO + k];
    sg[2][r][j] = sh[2][r][j] > 0.f ? s : 0.f;
  }
  __syncthreads();
  // layer 2: g2 = (g3 W3^T) * (h2 > 0)
  for (int e = tid; e < BR * NH; e += 256) {
    const int r = e / NH, j = e % NH;
    float s = 0.f;
#pragma unroll 16
    for (int k = 0; k < NH; ++k) s += sg[2][r][k] * params[OW3 + j * NH + k];
    sg[1][r][j] = sh[1][r][j] > 0.f ? s : 0.f;
  }
  __syncthreads();
  // layer 1: g1 = (g2 W2^T) * (h1 > 0)
  for (int e = tid; e < BR * NH; e += 256) {
    const int r = e / NH, j = e % NH;
    float s = 0.f;
#pragma unroll 16
    for (int k = 0; k < NH; ++k) s += sg[1][r][k] * params[OW2 + j * NH + k];
    sg[0][r][j] = sh[0][r][j] > 0.f ? s : 0.f;
  }
  __syncthreads();
  // parameter gradients: sums over the block's rows
  float* out = part + (int64_t)blockIdx.x * NPAR;
  for (int e = tid; e < NPAR; e += 256) {
    float s = 0.f;
    if (e < OB1) {  // W1[i][j] = sum x_i g1_j
      const int i = e / NH, j = e % NH;
      for (int r = 0; r < BR; ++r) s += sx[r][i] * sg[0][r][j];
    } else if (e < OW2) {
      const int j = e - OB1;
      for (int r = 0; r < BR; ++r) s += sg[0][r][j];
    } else if (e < OB2) {
      const int i = (e - OW2) / NH, j = (e - OW2) % NH;
      for (int r = 0; r < BR; ++r) s += sh[0][r][i] * sg[1][r][j];
    } else if (e < OW3) {
      const int j = e - OB2;
      for (int r = 0; r < BR; ++r) s += sg[1][r][j];
    } else if (e < OB3) {
      const int i = (e - OW3) / NH, j = (e - OW3) % NH;
      for (int r = 0; r < BR; ++r) s += sh[1][r][i] * sg[2][r][j];
    } else if (e < OW4) {
      const int j = e - OB3;
      for (int r = 0; r < BR; ++r) s += sg[2][r][j];
    } else if (e < OB4) {
      const int i = (e - OW4) / NO, j = (e - OW4) % NO;
      for (int r = 0; r < BR; ++r) s += sh[2][r][i] * se[r][j];
    } else {
      const int j = e - OB4;
      for (int r = 0; r < BR; ++r) s += se[r][j];
    }
    out[e] = s;
  }
}

__global__ void grad_reduce_kernel(int nblk, const float* __restrict__ part,
                                   float* __restrict__ grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NPAR) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += (double)part[(int64_t)b * NPAR + e];
  grad[e] = (float)s;
}

// -------------------------------------------------------------------- loss ----
// Groups of G = 1 + npos + nneg rows: query, exact neighbors, non-neighbors.
// d_j = |e_q - e_j|^2; loss = mean over (p, n) of softplus((d_p - d_n) / tau).
// One thread per group writes the loss and dE for all of the group's rows.
__global__ void pair_loss_kernel(int64_t groups, int npos, int nneg, float tau,
                                 const float* __restrict__ E, float* __restrict__ dE,
                                 float* __restrict__ loss) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= groups) return;
  const int G = 1 + npos + nneg;
  const float* eg = E + b * G * NO;
  float* dg = dE + b * G * NO;
  float q[NO];
#pragma unroll
  for (int k = 0; k < NO; ++k) q[k] = eg[k];
  // distances
  float d[128];
  for (int j = 1; j < G; ++j) {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < NO; ++k) {
      const float df = q[k] - eg[j * NO + k];
      s += df * df;
    }
    d[j - 1] = s;
  }
  const float scale = 1.f / (float)(npos * nneg);
  float gd[128];
  for (int j = 0; j < G - 1; ++j) gd[j] = 0.f;
  float L = 0.f;
  for (int p = 0; p < npos; ++p)
    for (int n2 = 0; n2 < nneg; ++n2) {
      const float z = (d[p] - d[npos + n2]) / tau;
      // softplus and logistic, overflow-safe
      const float sp = z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z));
      const float sg = z > 0.f ? 1.f / (1.f + expf(-z)) : expf(z) / (1.f + expf(z));
      L += sp;
      const float w = sg * scale / tau;
      gd[p] += w;
      gd[npos + n2] -= w;
    }
  loss[b] = L * scale;
  float gq[NO];
#pragma unroll
  for (int k = 0; k < NO; ++k) gq[k] = 0.f;
  for (int j = 1; j < G; ++j) {
    const float w = 2.f * gd[j - 1];
#pragma unroll
    for (int k = 0; k < NO; ++k) {
      const float df = q[k] - eg[j * NO + k];
      gq[k] += w * df;
      dg[j * NO + k] = -w * df;
    }
  }
#pragma unroll
  for (int k = 0; k < NO; ++k) dg[k] = gq[k];
}

// -------------------------------------------------------------------- Adam ----
__global__ void adam_kernel(int64_t count, float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------ batch build ----
// Rows of a training batch: for query q, [q, its npos exact neighbors, the
// exact list's next nhard entries (ranks npos .. npos+nhard-1), nrand earlier
// points drawn from the index window [q - rand_window, q)]; features gathered.
// A random draw that hits one of the query's listed points takes the last hard
// negative instead.
__global__ void batch_kernel(int64_t nq, const int32_t* __restrict__ queries,
                             const int32_t* __restrict__ nbr_ext, int m_ext, int npos, int nhard,
                             int nrand, const uint32_t* __restrict__ rnd, int rand_window,
                             const float* __restrict__ X, float* __restrict__ Xb) {
  const int G = 1 + npos + nhard + nrand;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nq * G) return;
  const int64_t b = e / G;
  const int slot = (int)(e - b * G);
  const int32_t q = queries[b];
  const int32_t* row = nbr_ext + (int64_t)q * m_ext;
  int32_t j;
  if (slot == 0) {
    j = q;
  } else if (slot <= npos + nhard) {
    j = row[slot - 1];
  } else {
    const uint32_t u = rnd[b * nrand + (slot - 1 - npos - nhard)];
    const int w = q < rand_window ? q : rand_window;
    j = q - 1 - (int32_t)(u % (uint32_t)w);
    for (int r = 0; r < npos + nhard; ++r)
      if (row[r] == j) j = row[npos + nhard - 1];
  }
#pragma unroll
  for (int c = 0; c < NI; ++c) Xb[e * NI + c] = X[(int64_t)j * NI + c];
}

}  // namespace

hipError_t launch_features(int64_t n, const double* sx, const double* sy, const double* t,
                           const FeatArgs& f, float* X, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, sx,
                     sy, t, f, X);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(int64_t rows, const float* params, const float* X, float* E,
                              float* H, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s,
                     rows, params, X, E, H);
  return hipGetLastError();
}

int64_t mlp_backward_blocks(int64_t rows) { return (rows + BR - 1) / BR; }

hipError_t launch_mlp_backward(int64_t rows, const float* params, const float* X, const float* H,
                               const float* dE, float* part, float* grad, hipStream_t s) {
  const int64_t nblk = mlp_backward_blocks(rows);
  if (nblk > 0)
    hipLaunchKernelGGL(mlp_backward_kernel, dim3((unsigned)nblk), dim3(256), 0, s, rows, params,
                       X, H, dE, part);
  hipLaunchKernelGGL(grad_reduce_kernel, dim3((NPAR + 255) / 256), dim3(256), 0, s, (int)nblk,
                     (const float*)part, grad);
  return hipGetLastError();
}

hipError_t launch_pair_loss(int64_t groups, int npos, int nneg, float tau, const float* E,
                            float* dE, float* loss, hipStream_t s) {
  if (groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(pair_loss_kernel, dim3((unsigned)((groups + 63) / 64)), dim3(64), 0, s,
                     groups, npos, nneg, tau, E, dE, loss);
  return hipGetLastError();
}

hipError_t launch_adam(int64_t count, float* p, const float* g, float* m, float* v, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count,
                     p, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_batch(int64_t nq, const int32_t* queries, const int32_t* nbr_ext, int m_ext,
                        int npos, int nhard, int nrand, const uint32_t* rnd, int rand_window,
                        const float* X, float* Xb, hipStream_t s) {
  const int64_t tot = nq * (1 + npos + nhard + nrand);
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, nq,
                     queries, nbr_ext, m_ext, npos, nhard, nrand, rnd, rand_window, X, Xb);
  return hipGetLastError();
}

}  // namespace vif
