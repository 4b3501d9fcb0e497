// Kernels of the learned warm start's network: a multilayer perceptron with silu
// hidden layers, trained by Adam on normalised targets.
//
// Weights live in FP32 (master copy, Adam moments) and are read by the passes as
// bfloat16 (round to nearest even), halving their footprint; activations and
// gradients are FP32 and every product accumulates in FP32.  Every product is one
// tiled GEMM on the BF16 matrix cores (v_mfma_f32_16x16x16_bf16): an FP32 operand
// enters as the exact sum of three bfloat16 terms (x = h + m + l; each remainder
// after rounding to the nearest bfloat16 is exact in FP32 and has at most 16, then
// 8, significant bits), a bfloat16 weight as itself.  Each term product is exact in
// FP32; against bfloat16 weights the three term products give the FP32 operand's
// product exactly, and between two FP32 operands the six term products of order
// up to 2^-16 are taken (the three dropped ones are below 2^-23 of the product).
// The bias, silu and silu' factors are fused into the epilogue:
#include <algorithm>

#include "mlp.h"

namespace vemb {
namespace {

constexpr int BM = 64, BN = 64, BK = 16, GT = 256;
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline float load_b(const float* p, long i) { return p[i]; }
__device__ inline float load_b(const uint16_t* p, long i) { return bf16_to_f32(p[i]); }

// x = t[0] + t[1] + t[2] exactly (finite x whose rounding stays finite); a non-finite
// leading term carries x alone.
__device__ inline void split3(float x, short t[3]) {
  const uint16_t h = f32_to_bf16(x);
  const float fh = bf16_to_f32(h);
  t[0] = (short)h;
  if (!isfinite(fh)) {
    t[1] = t[2] = 0;
    return;
  }
  const float r1 = x - fh;
  const uint16_t m = f32_to_bf16(r1);
  t[1] = (short)m;
  t[2] = (short)f32_to_bf16(r1 - bf16_to_f32(m));
}

__device__ inline float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ inline float silu(float z) { return z * sigm(z); }
__device__ inline float silu_grad(float z) {
  const float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}

// 64 x 64 output tile per workgroup, four wavefronts of 32 x 32 (2 x 2 MFMA tiles
// of 16 x 16), K staged through LDS (FP32) in steps of 16, one 16x16x16 product per
// term pair and step.  Lane layout of v_mfma_f32_16x16x16_bf16: lane l supplies
// A(l % 16, 4 (l / 16) + v) and B(4 (l / 16) + v, l % 16) as element v of its four;
// result D(i, j) in lane j + 16 (i / 4), register i % 4.
__device__ inline void epilogue(const GemmArgs& g, int i, int j, float v) {
  if (g.bias) v += g.bias[j];
  const long o = (long)i * g.ldc + j;
  if (g.epi == kEpiSilu) {
    g.C[o] = v;
    g.C2[o] = silu(v);
  } else if (g.epi == kEpiSiluGrad) {
    g.C[o] = v * silu_grad(g.Z[(long)i * g.ldz + j]);
  } else {
    g.C[o] = v;
  }
}

template <typename TB>
__global__ void __launch_bounds__(GT) gemm_kernel(GemmArgs g) {
  constexpr bool kBf16B = sizeof(TB) == 2;
  __shared__ float As[BK][BM + 4];
  __shared__ float Bs[BK][BN + 4];
  const TB* B = static_cast<const TB*>(g.B);
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  const bool a_kfast = g.sak == 1;  // choose the thread mapping that reads contiguous memory
  const bool b_jfast = g.sbj == 1;
  const int kbeg = blockIdx.z * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int r = 0; r < (BM * BK) / GT; ++r) {
      const int idx = tid + r * GT;
      int i, k;
      if (a_kfast) {
        k = idx % BK;
        i = idx / BK;
      } else {
        i = idx % BM;
        k = idx / BM;
      }
      const int gi = m0 + i, gk = k0 + k;
      As[k][i] = (gi < g.M && gk < kend) ? g.A[(long)gi * g.sai + (long)gk * g.sak] : 0.f;
    }
#pragma unroll
    for (int r = 0; r < (BN * BK) / GT; ++r) {
      const int idx = tid + r * GT;
      int j, k;
      if (b_jfast) {
        j = idx % BN;
        k = idx / BN;
      } else {
        k = idx % BK;
        j = idx / BK;
      }
      const int gj = n0 + j, gk = k0 + k;
      Bs[k][j] = (gj < g.N && gk < kend) ? load_b(B, (long)gk * g.sbk + (long)gj * g.sbj) : 0.f;
    }
    __syncthreads();
    // bfloat16 terms of this lane's four A and four B entries per 16-column tile
    constexpr int SB = kBf16B ? 1 : 3;
    s4 at[2][3], bt[2][SB];
    const int kq = 4 * (lane >> 4);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        short ta[3];
        split3(As[kq + v][wm + t * 16 + (lane & 15)], ta);
#pragma unroll
        for (int q = 0; q < 3; ++q) at[t][q][v] = ta[q];
        const float b = Bs[kq + v][wn + t * 16 + (lane & 15)];
        if constexpr (kBf16B) {
          bt[t][0][v] = (short)(__float_as_uint(b) >> 16);  // a widened bfloat16: exact
        } else {
          short tb[3];
          split3(b, tb);
#pragma unroll
          for (int q = 0; q < 3; ++q) bt[t][q][v] = tb[q];
        }
      }
    // term pairs of order <= 2^-16, smallest first
#pragma unroll
    for (int ord = 2; ord >= 0; --ord)
#pragma unroll
      for (int qa = 0; qa <= ord; ++qa) {
        const int qb = ord - qa;
        if (qb >= SB) continue;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(at[a][qa], bt[b][qb], acc[a][b], 0, 0, 0);
      }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm + a * 16 + 4 * (lane >> 4) + r;
        const int j = n0 + wn + b * 16 + (lane & 15);
        if (i < g.M && j < g.N) {
          if (g.splits > 1)
            g.ws[((long)blockIdx.z * g.M + i) * g.N + j] = acc[a][b][r];
          else
            epilogue(g, i, j, acc[a][b][r]);
        }
      }
}

// Sum of the split-K partial tiles (fixed order) and the epilogue.
__global__ void __launch_bounds__(256) splitk_reduce_kernel(GemmArgs g) {
  const long MN = (long)g.M * g.N;
  for (long idx = blockIdx.x * 256L + threadIdx.x; idx < MN; idx += (long)gridDim.x * 256) {
    float v = 0.f;
    for (int z = 0; z < g.splits; ++z) v += g.ws[z * MN + idx];
    epilogue(g, (int)(idx / g.N), (int)(idx % g.N), v);
  }
}

// dY = 2 (Y - (T - mean)/std) / (B O); per-block partial sums of the squared residual.
__global__ void __launch_bounds__(256) loss_grad_kernel(const float* Y, const float* T, const float* mean,
                                                        const float* stdv, long B, int O, float* dY,
                                                        double* partial) {
  __shared__ double red[256];
  const long total = B * O;
  const double scale = 2.0 / (double)total;
  double acc = 0.0;
  for (long idx = blockIdx.x * 256L + threadIdx.x; idx < total; idx += (long)gridDim.x * 256) {
    const int j = (int)(idx % O);
    const float th = (T[idx] - mean[j]) / stdv[j];
    const float r = Y[idx] - th;
    dY[idx] = (float)(scale * r);
    acc += (double)r * r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) sum_partials_kernel(const double* partial, int n, double scale, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0] * scale;
}

// db_j = sum_b dZ(b, j)
__global__ void __launch_bounds__(256) colsum_kernel(const float* dZ, int B, int N, float* db) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  float acc = 0.f;
  for (int b = 0; b < B; ++b) acc += dZ[(long)b * N + j];
  db[j] = acc;
}

// Adam on the flat FP32 parameters; refreshes the bfloat16 copy read by the passes.
__global__ void __launch_bounds__(256) adam_kernel(float* theta, float* m, float* v, const float* g, uint16_t* wbf,
                                                   long n, float lr, float c1, float c2) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = kAdamB1 * m[i] + (1.f - kAdamB1) * gi;
    const float vi = kAdamB2 * v[i] + (1.f - kAdamB2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float th = theta[i] - lr * (mi * c1) / (sqrtf(vi * c2) + kAdamEps);
    theta[i] = th;
    wbf[i] = f32_to_bf16(th);
  }
}

__global__ void __launch_bounds__(256) to_bf16_kernel(const float* theta, uint16_t* wbf, long n) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) wbf[i] = f32_to_bf16(theta[i]);
}

// Per-column mean and standard deviation (FP64 sums), unfloored.
__global__ void __launch_bounds__(256) colstats_kernel(const float* T, int count, int O, float* mean, float* stdv) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= O) return;
  double s = 0.0;
  for (int b = 0; b < count; ++b) s += T[(long)b * O + j];
  const double mu = s / count;
  double q = 0.0;
  for (int b = 0; b < count; ++b) {
    const double d = T[(long)b * O + j] - mu;
    q += d * d;
  }
  mean[j] = (float)mu;
  stdv[j] = (float)sqrt(q / count);
}

// std_j <- max(std_j, max(floor_abs, rel * max_j std_j)); one workgroup.
__global__ void __launch_bounds__(256) std_floor_kernel(float* stdv, int O, float floor_abs, float rel) {
  __shared__ float red[256];
  float v = 0.f;
  for (int j = threadIdx.x; j < O; j += 256) v = fmaxf(v, stdv[j]);
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const float fl = fmaxf(floor_abs, rel * red[0]);
  for (int j = threadIdx.x; j < O; j += 256) stdv[j] = fmaxf(stdv[j], fl);
}

__global__ void __launch_bounds__(256) denorm_kernel(const float* Y, const float* mean, const float* stdv, long B,
                                                     int O, float* out) {
  const long total = B * O;
  for (long idx = blockIdx.x * 256L + threadIdx.x; idx < total; idx += (long)gridDim.x * 256) {
    const int j = (int)(idx % O);
    out[idx] = Y[idx] * stdv[j] + mean[j];
  }
}

// Gather rows[b] of X (count x d) into dst (B x d); rows out of range give zeros.
__global__ void __launch_bounds__(256) gather_rows_kernel(const float* X, int count, const int* rows, int B, int d,
                                                          float* dst) {
  const long total = (long)B * d;
  for (long idx = blockIdx.x * 256L + threadIdx.x; idx < total; idx += (long)gridDim.x * 256) {
    const long b = idx / d, c = idx - b * d;
    const int r = rows[b];
    dst[idx] = (r >= 0 && r < count) ? X[(long)r * d + c] : 0.f;
  }
}

int grid_for(long total) {
  const long g = (total + 255) / 256;
  return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

}  // namespace

hipError_t launch_gemm(const GemmArgs& g_in, bool b_is_bf16, hipStream_t st) {
  GemmArgs g = g_in;
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int gx = (g.N + BN - 1) / BN, gy = (g.M + BM - 1) / BM;
  // split K when there are few output tiles and a long reduction
  int splits = 1;
  if (g.ws && gx * gy < 128 && g.K >= 1024) {
    splits = std::min(256 / (gx * gy) + 1, g.K / 256);
    const long cap = g.ws_floats / ((long)g.M * g.N);
    if (splits > cap) splits = (int)cap;
    if (splits < 2) splits = 1;
  }
  g.splits = splits;
  g.kchunk = ((g.K + splits - 1) / splits + BK - 1) / BK * BK;
  if (splits > 1) g.splits = (g.K + g.kchunk - 1) / g.kchunk;
  dim3 grid(gx, gy, g.splits);
  if (b_is_bf16)
    hipLaunchKernelGGL(gemm_kernel<uint16_t>, grid, dim3(GT), 0, st, g);
  else
    hipLaunchKernelGGL(gemm_kernel<float>, grid, dim3(GT), 0, st, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g.splits == 1) return e;
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid_for((long)g.M * g.N)), dim3(256), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_loss_grad(const float* Y, const float* T, const float* mean, const float* stdv, int B, int O,
                            float* dY, double* partial, int max_partials, double* loss, hipStream_t st) {
  const long total = (long)B * O;
  int blocks = grid_for(total);
  if (blocks > max_partials) blocks = max_partials;
  hipLaunchKernelGGL(loss_grad_kernel, dim3(blocks), dim3(256), 0, st, Y, T, mean, stdv, (long)B, O, dY, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, st, partial, blocks, 1.0 / (double)total, loss);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* dZ, int B, int N, float* db, hipStream_t st) {
  hipLaunchKernelGGL(colsum_kernel, dim3((N + 255) / 256), dim3(256), 0, st, dZ, B, N, db);
  return hipGetLastError();
}

hipError_t launch_adam(float* theta, float* m, float* v, const float* g, uint16_t* wbf, long n, float lr, float c1,
                       float c2, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, st, theta, m, v, g, wbf, n, lr, c1, c2);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* theta, uint16_t* wbf, long n, hipStream_t st) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, st, theta, wbf, n);
  return hipGetLastError();
}

hipError_t launch_colstats(const float* T, int count, int O, float* mean, float* stdv, float floor_abs, float rel,
                           hipStream_t st) {
  hipLaunchKernelGGL(colstats_kernel, dim3((O + 255) / 256), dim3(256), 0, st, T, count, O, mean, stdv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(std_floor_kernel, dim3(1), dim3(256), 0, st, stdv, O, floor_abs, rel);
  return hipGetLastError();
}

hipError_t launch_denorm(const float* Y, const float* mean, const float* stdv, int B, int O, float* out,
                         hipStream_t st) {
  hipLaunchKernelGGL(denorm_kernel, dim3(grid_for((long)B * O)), dim3(256), 0, st, Y, mean, stdv, (long)B, O, out);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const float* X, int count, const int* rows, int B, int d, float* dst, hipStream_t st) {
  hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_for((long)B * d)), dim3(256), 0, st, X, count, rows, B, d, dst);
  return hipGetLastError();
}

}  // namespace vemb
