// Kernels of the learned Davidson preconditioner: features, the fused FP32
// MLP forward (inference and training), backward elementwise parts, column
// sums and Adam.  The training GEMMs reuse the grouped GEMM kernel (FP32).
//
// Forward tile: one workgroup (256 threads = 4 waves) evaluates 64 elements.
// Thread t owns output columns 4*(t%64) .. +3 for the 16 elements 16*(t/64) ..
// +15 (so every wave owns 16 elements and all 256 columns): layer 1 and layer
// 2 are register-blocked FMA loops over a transposed activation tile in LDS,
// and layer 3 is a wave reduction across the 64 column groups.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/dmrg.h"
#include "common.h"
#include "device.h"

namespace dmrg {

namespace {
inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }
constexpr int NF = DMRG_MLP_NFEAT, HD = DMRG_MLP_HIDDEN, TE = 64;
static_assert(HD == 256, "forward tile assumes 256 hidden units");

struct WPtr {
  const float *W1, *b1, *W2, *b2, *w3, *b3;
};
__device__ __forceinline__ WPtr wptr(const float* w) {
  WPtr p;
  p.W1 = w;
  p.b1 = p.W1 + NF * HD;
  p.W2 = p.b1 + HD;
  p.b2 = p.W2 + HD * HD;
  p.w3 = p.b2 + HD;
  p.b3 = p.w3 + HD;
  return p;
}

// 64 elements: F[64][NF] in LDS -> g[64] in LDS.  a1/a2 (optional, global,
// row-major [row0 + e][HD]) receive the post-ReLU activations of rows < nrow.
__device__ void forward_tile(const float (*F)[NF + 1], float (*H1T)[TE + 4], float* gout, const float* w,
                             float* a1, float* a2, int64_t row0, int nrow) {
  const WPtr P = wptr(w);
  const int t = threadIdx.x, c = t & 63, eg = (t >> 6) * 16;
  // layer 1
  float acc[16][4];
  {
    const float4 bb = *reinterpret_cast<const float4*>(P.b1 + 4 * c);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      acc[e][0] = bb.x;
      acc[e][1] = bb.y;
      acc[e][2] = bb.z;
      acc[e][3] = bb.w;
    }
    for (int f = 0; f < NF; ++f) {
      const float4 wv = *reinterpret_cast<const float4*>(P.W1 + f * HD + 4 * c);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const float x = F[eg + e][f];
        acc[e][0] += x * wv.x;
        acc[e][1] += x * wv.y;
        acc[e][2] += x * wv.z;
        acc[e][3] += x * wv.w;
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float v = acc[e][j] > 0.f ? acc[e][j] : 0.f;
        H1T[4 * c + j][eg + e] = v;
        if (a1 && eg + e < nrow) a1[(row0 + eg + e) * HD + 4 * c + j] = v;
      }
  }
  __syncthreads();
  // layer 2
  {
    const float4 bb = *reinterpret_cast<const float4*>(P.b2 + 4 * c);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      acc[e][0] = bb.x;
      acc[e][1] = bb.y;
      acc[e][2] = bb.z;
      acc[e][3] = bb.w;
    }
    for (int k = 0; k < HD; ++k) {
      const float4 wv = *reinterpret_cast<const float4*>(P.W2 + k * HD + 4 * c);
      float h[16];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 hv = *reinterpret_cast<const float4*>(&H1T[k][eg + 4 * q]);
        h[4 * q] = hv.x;
        h[4 * q + 1] = hv.y;
        h[4 * q + 2] = hv.z;
        h[4 * q + 3] = hv.w;
      }
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        acc[e][0] += h[e] * wv.x;
        acc[e][1] += h[e] * wv.y;
        acc[e][2] += h[e] * wv.z;
        acc[e][3] += h[e] * wv.w;
      }
    }
  }
  // layer 3: partial dot with w3 over this thread's 4 columns, then a wave
  // reduction over the 64 column groups (fixed butterfly order)
  const float4 w3 = *reinterpret_cast<const float4*>(P.w3 + 4 * c);
  float part[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float v = acc[e][j] > 0.f ? acc[e][j] : 0.f;
      if (a2 && eg + e < nrow) a2[(row0 + eg + e) * HD + 4 * c + j] = v;
      s += v * (j == 0 ? w3.x : j == 1 ? w3.y : j == 2 ? w3.z : w3.w);
    }
    part[e] = s;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int e = 0; e < 16; ++e) part[e] += __shfl_xor(part[e], off, 64);
  if (c == 0) {
    const float b3 = *P.b3;
#pragma unroll
    for (int e = 0; e < 16; ++e) gout[eg + e] = part[e] + b3;
  }
  __syncthreads();
}

__device__ __forceinline__ float clampf(float x, float lo, float hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Features of element i (see dmrg.h); blk[i] is its psi block, stat[b][14]
// the block's static features (columns 4..17).
__device__ void features(int64_t i, const double* r, const double* diag, double theta, const double* scales,
                         const int* blk, const float* stat, float* f) {
  const double dh = diag[i] - theta;
  const float sh = (float)scales[0], sr = (float)scales[1];
  f[0] = clampf((float)dh / sh, -8.f, 8.f);
  f[1] = asinhf((float)(dh / scales[2])) / 4.f;
  f[2] = clampf((float)r[i] / sr, -8.f, 8.f);
  f[3] = (float)log10(scales[2]) / 4.f;
  const float* s = stat + (int64_t)blk[i] * (NF - 4);
#pragma unroll
  for (int j = 0; j < NF - 4; ++j) f[4 + j] = s[j];
}

__device__ __forceinline__ double diag_corr(double r, double dg, double theta, double fl) {
  double den = theta - dg;
  if (fabs(den) < fl) den = den < 0 ? -fl : fl;
  return r / den;
}

// t_i = g(f_i) * r_i / (theta - H_ii) for all i
__global__ __launch_bounds__(256) void mlp_apply_kernel(const float* w, const double* r, const double* diag,
                                                        const double* theta_p, const double* scales,
                                                        const int* blk, const float* stat, double fl, double* out,
                                                        int64_t n) {
  __shared__ float F[TE][NF + 1];
  __shared__ float H1T[HD][TE + 4];
  __shared__ float g[TE];
  const double theta = *theta_p;
  for (int64_t base = (int64_t)blockIdx.x * TE; base < n; base += (int64_t)gridDim.x * TE) {
    const int t = threadIdx.x;
    if (t < TE) {
      const int64_t i = base + t;
      if (i < n)
        features(i, r, diag, theta, scales, blk, stat, F[t]);
      else
        for (int j = 0; j < NF; ++j) F[t][j] = 0.f;
    }
    __syncthreads();
    forward_tile(F, H1T, g, w, nullptr, nullptr, 0, 0);
    if (t < TE && base + t < n) {
      const int64_t i = base + t;
      out[i] = (double)g[t] * diag_corr(r[i], diag[i], theta, fl);
    }
    __syncthreads();
  }
}

// sums of (diag - theta)^2 and r^2: fixed-order partial sums, then one block
constexpr int SC_CHUNKS = 256;
__global__ void scales_partial(const double* r, const double* diag, const double* theta_p, int64_t n,
                               double* part) {
  const double theta = *theta_p;
  const int64_t per = (n + SC_CHUNKS - 1) / SC_CHUNKS;
  const int64_t b = blockIdx.x * per, e = b + per < n ? b + per : n;
  double s0 = 0, s1 = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    const double dh = diag[i] - theta;
    s0 += dh * dh;
    s1 += r[i] * r[i];
  }
  __shared__ double red[2][256];
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}
__global__ void scales_final(const double* part, int64_t n, double* scales) {
  if (threadIdx.x == 0) {
    double s0 = 0, s1 = 0;
    for (int c = 0; c < SC_CHUNKS; ++c) {
      s0 += part[2 * c];
      s1 += part[2 * c + 1];
    }
    const double tiny = 1e-300;
    scales[0] = sqrt(s0 / (double)n) + tiny;
    scales[1] = sqrt(s1 / (double)n) + tiny;
    scales[2] = sqrt(s1) + tiny;
  }
}

// features, d_i and target at sampled indices
__global__ void gather_pairs_kernel(const int64_t* idx, int m, const double* r, const double* diag,
                                    const double* theta_p, const double* scales, const int* blk, const float* stat,
                                    const double* e, double es, double fl, float* feat, float* dcorr,
                                    float* target) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int64_t i = idx[j];
  const double theta = *theta_p;
  float f[NF];
  features(i, r, diag, theta, scales, blk, stat, f);
  for (int q = 0; q < NF; ++q) feat[(int64_t)j * NF + q] = f[q];
  dcorr[j] = (float)diag_corr(r[i], diag[i], theta, fl);
  target[j] = (float)(es * e[i]);
}

// training forward over rows [0, n) of F (global [n][NF])
__global__ __launch_bounds__(256) void mlp_train_fwd_kernel(const float* w, const float* Fg, int64_t n, float* a1,
                                                            float* a2, float* gout) {
  __shared__ float F[TE][NF + 1];
  __shared__ float H1T[HD][TE + 4];
  __shared__ float g[TE];
  for (int64_t base = (int64_t)blockIdx.x * TE; base < n; base += (int64_t)gridDim.x * TE) {
    const int t = threadIdx.x;
    const int nrow = (int)(n - base < TE ? n - base : TE);
    if (t < TE)
      for (int j = 0; j < NF; ++j) F[t][j] = t < nrow ? Fg[(base + t) * NF + j] : 0.f;
    __syncthreads();
    forward_tile(F, H1T, g, w, a1, a2, base, nrow);
    if (t < nrow) gout[base + t] = g[t];
    __syncthreads();
  }
}

// dout = 2 (g d - y) d / n ;  dz2 = dout w3 [a2 > 0]
__global__ void mlp_bwd_out_kernel(const float* w, const float* g, const float* d, const float* y, const float* a2,
                                   int64_t n, float* dout, float* dz2) {
  const WPtr P = wptr(w);
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n * HD; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = k / HD;
    const int j = (int)(k % HD);
    const float o = 2.f * (g[b] * d[b] - y[b]) * d[b] / (float)n;
    if (j == 0) dout[b] = o;
    dz2[k] = a2[k] > 0.f ? o * P.w3[j] : 0.f;
  }
}

// Direction loss of one group (the samples of one Davidson iteration):
// L = 1 - <t,y>^2 / (<t,t> <y,y>) with t_b = g_b d_b.  One block computes the
// three sums in a fixed order, then dL/dg_b = (dL/dt_b) d_b and
// dz2 = dL/dg w3 [a2 > 0]; loss[0] receives L.
__global__ void mlp_cos_grad_kernel(const float* w, const float* g, const float* d, const float* y, const float* a2,
                                    int64_t n, float* dout, float* dz2, float* loss) {
  __shared__ float red[3][256];
  float A = 0.f, T = 0.f, Y = 0.f;
  for (int64_t b = threadIdx.x; b < n; b += blockDim.x) {
    const float t = g[b] * d[b];
    A += t * y[b];
    T += t * t;
    Y += y[b] * y[b];
  }
  red[0][threadIdx.x] = A;
  red[1][threadIdx.x] = T;
  red[2][threadIdx.x] = Y;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
    __syncthreads();
  }
  A = red[0][0];
  T = red[1][0] + 1e-30f;
  Y = red[2][0] + 1e-30f;
  if (threadIdx.x == 0) *loss = 1.f - A * A / (T * Y);
  const WPtr P = wptr(w);
  for (int64_t k = threadIdx.x; k < n * HD; k += blockDim.x) {
    const int64_t b = k / HD;
    const int j = (int)(k % HD);
    const float t = g[b] * d[b];
    const float o = (-2.f * A * y[b] / (T * Y) + 2.f * A * A * t / (T * T * Y)) * d[b];
    if (j == 0) dout[b] = o;
    dz2[k] = a2[k] > 0.f ? o * P.w3[j] : 0.f;
  }
}

__global__ void relu_mask_kernel(float* dz, const float* a, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    if (!(a[k] > 0.f)) dz[k] = 0.f;
}

// out[j] = sum_b X[b][j] * (v ? v[b] : 1), columns j < ncol (fixed order)
__global__ void colsum_kernel(const float* X, const float* v, int64_t n, int ncol, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncol) return;
  float s = 0.f;
  for (int64_t b = 0; b < n; ++b) s += X[b * ncol + j] * (v ? v[b] : 1.f);
  out[j] = s;
}

__global__ void sum_kernel(const float* x, int64_t n, float* out) {
  __shared__ float red[256];
  float s = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void adam_kernel(float* w, const float* gr, float* m, float* v, int64_t n, float lr, float b1, float b2,
                            float c1, float c2, float eps) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gg = gr[i];
    const float mm = b1 * m[i] + (1.f - b1) * gg;
    const float vv = b2 * v[i] + (1.f - b2) * gg * gg;
    m[i] = mm;
    v[i] = vv;
    w[i] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// squared error per row (for the reported loss)
__global__ void sqerr_kernel(const float* g, const float* d, const float* y, int64_t n, float* out) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < n; b += (int64_t)gridDim.x * blockDim.x) {
    const float e = g[b] * d[b] - y[b];
    out[b] = e * e;
  }
}

__global__ void gather_rows_kernel(const float* src, const int* perm, int64_t n, int width, float* dst) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n * width; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = k / width;
    dst[k] = src[(int64_t)perm[b] * width + k % width];
  }
}

inline unsigned grid_for(int64_t work, int per = 256, int64_t cap = 65536) {
  int64_t b = (work + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}
}  // namespace

void k_mlp_scales(const double* r, const double* diag, const double* theta, int64_t n, double* part,
                  double* scales, void* s) {
  hipLaunchKernelGGL(scales_partial, dim3(SC_CHUNKS), dim3(256), 0, S(s), r, diag, theta, n, part);
  hipLaunchKernelGGL(scales_final, dim3(1), dim3(64), 0, S(s), part, n, scales);
  dev_check("k_mlp_scales");
}

void k_mlp_apply(const float* w, const double* r, const double* diag, const double* theta, const double* scales,
                 const int* blk, const float* stat, double fl, double* out, int64_t n, void* s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(mlp_apply_kernel, dim3(grid_for(n, TE, 8192)), dim3(256), 0, S(s), w, r, diag, theta, scales,
                     blk, stat, fl, out, n);
  dev_check("k_mlp_apply");
}

void k_mlp_gather_pairs(const int64_t* idx, int m, const double* r, const double* diag, const double* theta,
                        const double* scales, const int* blk, const float* stat, const double* e, double es, double fl,
                        float* feat, float* dcorr, float* target, void* s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(gather_pairs_kernel, dim3((m + 127) / 128), dim3(128), 0, S(s), idx, m, r, diag, theta, scales,
                     blk, stat, e, es, fl, feat, dcorr, target);
  dev_check("k_mlp_gather_pairs");
}

void k_mlp_train_fwd(const float* w, const float* F, int64_t n, float* a1, float* a2, float* g, void* s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(mlp_train_fwd_kernel, dim3(grid_for(n, TE, 8192)), dim3(256), 0, S(s), w, F, n, a1, a2, g);
  dev_check("k_mlp_train_fwd");
}

void k_mlp_bwd_out(const float* w, const float* g, const float* d, const float* y, const float* a2, int64_t n,
                   float* dout, float* dz2, void* s) {
  hipLaunchKernelGGL(mlp_bwd_out_kernel, dim3(grid_for(n * HD)), dim3(256), 0, S(s), w, g, d, y, a2, n, dout, dz2);
  dev_check("k_mlp_bwd_out");
}

void k_mlp_cos_grad(const float* w, const float* g, const float* d, const float* y, const float* a2, int64_t n,
                    float* dout, float* dz2, float* loss, void* s) {
  hipLaunchKernelGGL(mlp_cos_grad_kernel, dim3(1), dim3(256), 0, S(s), w, g, d, y, a2, n, dout, dz2, loss);
  dev_check("k_mlp_cos_grad");
}

void k_relu_mask(float* dz, const float* a, int64_t n, void* s) {
  hipLaunchKernelGGL(relu_mask_kernel, dim3(grid_for(n)), dim3(256), 0, S(s), dz, a, n);
  dev_check("k_relu_mask");
}

void k_colsum(const float* X, const float* v, int64_t n, int ncol, float* out, void* s) {
  hipLaunchKernelGGL(colsum_kernel, dim3((ncol + 63) / 64), dim3(64), 0, S(s), X, v, n, ncol, out);
  dev_check("k_colsum");
}

void k_sum_f(const float* x, int64_t n, float* out, void* s) {
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, S(s), x, n, out);
  dev_check("k_sum_f");
}

void k_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float c1, float c2,
            float eps, void* s) {
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, S(s), w, g, m, v, n, lr, b1, b2, c1, c2, eps);
  dev_check("k_adam");
}

void k_sqerr(const float* g, const float* d, const float* y, int64_t n, float* out, void* s) {
  hipLaunchKernelGGL(sqerr_kernel, dim3(grid_for(n)), dim3(256), 0, S(s), g, d, y, n, out);
  dev_check("k_sqerr");
}

void k_gather_rows(const float* src, const int* perm, int64_t n, int width, float* dst, void* s) {
  hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_for(n * width)), dim3(256), 0, S(s), src, perm, n, width, dst);
  dev_check("k_gather_rows");
}

}  // namespace dmrg
