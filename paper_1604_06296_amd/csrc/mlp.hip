// Multilayer perceptron for the loop surrogate: BF16 matrix-core GEMMs with
// FP32 accumulation and FP32 master weights, SiLU hidden layers, mean-squared
// loss, backpropagation and Adam, and the tufrg_mlp_* C ABI.
//
// Layer l: z_l = a_{l-1} W_l^T + b_l, a_l = silu(z_l) on hidden layers, a
// linear output.  Forward products use the BF16 hi/lo split of both operands
// (hi*hi + hi*lo + lo*hi, about 16 mantissa bits), so that predictions carry
// FP32-like accuracy; gradient products use plain BF16 operands.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "tufrg_internal.h"

namespace tufrg {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// v_mfma_f32_16x16x32_bf16 operands: lane l holds A[l%16][8(l/16)+j] and
// B[8(l/16)+j][l%16], j = 0..7 (eight consecutive k of an LDS row)
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_value(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}
__device__ __forceinline__ float sigmoidf_(float z) { return 1.0f / (1.0f + __expf(-z)); }

enum Epilogue {
  kStore = 0,        // C = acc (split-K partials)
  kBiasSilu = 1,     // Z = acc + bias; C = silu(Z); Z stored when Zs != null
  kBias = 2,         // C = acc + bias
  kDsilu = 3         // C = acc * silu'(Zp)
};

struct GemmArgs {
  const float* A;    // op(A) is M x K: A[m*lda + k], or A[k*lda + m] when transA
  const float* B;    // op(B) is K x N: B[k*ldb + n], or B[n*ldb + k] when transB
  float* C;          // C[m*ldc + n] (+ blockIdx.z * split_stride)
  const float* bias; // [N]
  float* Zs;         // [M][ldz]
  const float* Zp;   // [M][ldzp]
  int64_t split_stride;
  int lda, ldb, ldc, ldz, ldzp;
  int transA, transB;
  int M, N, K, kps;  // kps: K range of one split (multiple of 32)
  int epi;
};

constexpr int kTM = 64, kTN = 64, kKC = 32, kLDK = kKC + 8;   // LDS row stride in halfwords

// C tile 64 x 64 per block of 4 waves; each wave owns a 32 x 32 quarter as
// 2 x 2 tiles of v_mfma_f32_16x16x32_bf16 (one step per K chunk of 32).
// Operands are read as FP32, rounded to BF16 (and split hi/lo when
// PASSES == 3) into LDS.
// VEC: op(A) = A and op(B) = B^T with rows of K contiguous and 16-byte
// aligned (lda, ldb multiples of 4): each thread stages two 4-wide K quads of
// A and of B with one 16-byte load each and one 8-byte LDS store per BF16 quad.
template <int PASSES, bool VEC>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) unsigned short Ah[kTM * kLDK];
  __shared__ __attribute__((aligned(16))) unsigned short Bh[kTN * kLDK];
  __shared__ __attribute__((aligned(16))) unsigned short Al[PASSES == 3 ? kTM * kLDK : 4];
  __shared__ __attribute__((aligned(16))) unsigned short Bl[PASSES == 3 ? kTN * kLDK : 4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
  const int kb = blockIdx.z * g.kps, ke = min(g.K, kb + g.kps);
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // software pipeline: the next K chunk's operands are loaded into registers
  // while the current chunk is in the matrix cores, then split and staged
  float av[8], bv[8];
  const int vr = tid >> 3, vk = 4 * (tid & 7);   // VEC: rows vr + 32 i, K quad vk
  auto quad = [&](const float* row, bool ok, int gk, float* dst) {
    if (ok && gk + 4 <= ke) {
      const float4 q = *reinterpret_cast<const float4*>(row + gk);
      dst[0] = q.x;
      dst[1] = q.y;
      dst[2] = q.z;
      dst[3] = q.w;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) dst[j] = (ok && gk + j < ke) ? row[gk + j] : 0.f;
    }
  };
  auto load = [&](int k0) {
    if constexpr (VEC) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int gm = m0 + vr + 32 * i, gn = n0 + vr + 32 * i;
        quad(g.A + (size_t)(gm < g.M ? gm : 0) * g.lda, gm < g.M, k0 + vk, av + 4 * i);
        quad(g.B + (size_t)(gn < g.N ? gn : 0) * g.ldb, gn < g.N, k0 + vk, bv + 4 * i);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = tid + 256 * i;
        const int m = g.transA ? e % kTM : e / kKC;
        const int k = g.transA ? e / kTM : e % kKC;
        const int gm = m0 + m, gk = k0 + k;
        av[i] = (gm < g.M && gk < ke) ? (g.transA ? g.A[(size_t)gk * g.lda + gm] : g.A[(size_t)gm * g.lda + gk])
                                      : 0.f;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = tid + 256 * i;
        const int n = g.transB ? e / kKC : e % kTN;
        const int k = g.transB ? e % kKC : e / kTN;
        const int gn = n0 + n, gk = k0 + k;
        bv[i] = (gn < g.N && gk < ke) ? (g.transB ? g.B[(size_t)gn * g.ldb + gk] : g.B[(size_t)gk * g.ldb + gn])
                                      : 0.f;
      }
    }
  };
  auto store_quad = [&](const float* v, unsigned short* hi, unsigned short* lo) {
    bf16x4 qh, ql;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const unsigned short h = bf16_rne(v[j]);
      qh[j] = (short)h;
      ql[j] = (short)bf16_rne(v[j] - bf16_value(h));
    }
    *reinterpret_cast<bf16x4*>(hi) = qh;
    if constexpr (PASSES == 3) *reinterpret_cast<bf16x4*>(lo) = ql;
  };
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += kKC) {
    if constexpr (VEC) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = vr + 32 * i;
        store_quad(av + 4 * i, &Ah[r * kLDK + vk], &Al[PASSES == 3 ? r * kLDK + vk : 0]);
        store_quad(bv + 4 * i, &Bh[r * kLDK + vk], &Bl[PASSES == 3 ? r * kLDK + vk : 0]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = tid + 256 * i;
        const int m = g.transA ? e % kTM : e / kKC;
        const int k = g.transA ? e / kTM : e % kKC;
        const unsigned short h = bf16_rne(av[i]);
        Ah[m * kLDK + k] = h;
        if constexpr (PASSES == 3) Al[m * kLDK + k] = bf16_rne(av[i] - bf16_value(h));
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = tid + 256 * i;
        const int n = g.transB ? e / kKC : e % kTN;
        const int k = g.transB ? e % kKC : e / kTN;
        const unsigned short h = bf16_rne(bv[i]);
        Bh[n * kLDK + k] = h;
        if constexpr (PASSES == 3) Bl[n * kLDK + k] = bf16_rne(bv[i] - bf16_value(h));
      }
    }
    __syncthreads();
    if (k0 + kKC < ke) load(k0 + kKC);
    {
      // the chunk's 32 k in one v_mfma_f32_16x16x32_bf16 step per product
      const int kq = 8 * (lane >> 4);
      bf16x8 ah[2], bh[2], al[2], bl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = wm + 16 * i + (lane & 15);
        const int c = wn + 16 * i + (lane & 15);
        ah[i] = *reinterpret_cast<const bf16x8*>(&Ah[r * kLDK + kq]);
        bh[i] = *reinterpret_cast<const bf16x8*>(&Bh[c * kLDK + kq]);
        if constexpr (PASSES == 3) {
          al[i] = *reinterpret_cast<const bf16x8*>(&Al[r * kLDK + kq]);
          bl[i] = *reinterpret_cast<const bf16x8*>(&Bl[c * kLDK + kq]);
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if constexpr (PASSES == 3) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          }
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  float* C = g.C + (size_t)blockIdx.z * g.split_stride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + jj;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        const float v = acc[i][j][jj];
        float out;
        if (g.epi == kBiasSilu) {
          const float z = v + g.bias[n];
          if (g.Zs) g.Zs[(size_t)m * g.ldz + n] = z;
          out = z * sigmoidf_(z);
        } else if (g.epi == kBias) {
          out = v + g.bias[n];
        } else if (g.epi == kDsilu) {
          const float z = g.Zp[(size_t)m * g.ldzp + n];
          const float s = sigmoidf_(z);
          out = v * s * (1.0f + z * (1.0f - s));
        } else {
          out = v;
        }
        C[(size_t)m * g.ldc + n] = out;
      }
}

// out[i] = sum_s part[s * stride + i] in split order (deterministic)
__global__ void k_sum_splits(const float* __restrict__ part, int nsplit, int64_t stride, int64_t n,
                             float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float v = 0.f;
  for (int s = 0; s < nsplit; ++s) v += part[(size_t)s * stride + i];
  out[i] = v;
}

// Column sums of dZ [rows][N] over row chunks of 256: part[chunk][N]
__global__ void k_colsum_part(const float* __restrict__ dz, int rows, int N, float* __restrict__ part) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int r0 = blockIdx.y * 256, r1 = min(rows, r0 + 256);
  float v = 0.f;
  for (int r = r0; r < r1; ++r) v += dz[(size_t)r * N + n];
  part[(size_t)blockIdx.y * N + n] = v;
}

// residual r = a - y; delta = 2 r / (rows * nout); per-block sum of r^2
__global__ void __launch_bounds__(256)
k_loss(const float* __restrict__ a, const float* __restrict__ y, int64_t n, float scale,
       float* __restrict__ delta, double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double s = 0.0;
  if (i < n) {
    const float r = a[i] - y[i];
    delta[i] = scale * r;
    s = (double)r * (double)r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_double(const double* __restrict__ part, int n, double scale, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  *out = s * scale;
}

// Adam with bias correction (Kingma & Ba 2015)
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

// minibatch rows drawn with replacement: row i of step s = hash(seed, s, i) mod n
__global__ void k_gather_rows(const float* __restrict__ x, int nin, const float* __restrict__ y, int nout,
                              int64_t n, int rows, uint64_t seed, uint64_t step, float* __restrict__ xb,
                              float* __restrict__ yb) {
  const int r = blockIdx.x;
  if (r >= rows) return;
  const uint64_t h = splitmix64(seed ^ splitmix64(step * 0x100000001b3ull + (uint64_t)r));
  const int64_t src = (int64_t)(h % (uint64_t)n);
  for (int c = threadIdx.x; c < nin; c += blockDim.x) xb[(size_t)r * nin + c] = x[(size_t)src * nin + c];
  for (int c = threadIdx.x; c < nout; c += blockDim.x) yb[(size_t)r * nout + c] = y[(size_t)src * nout + c];
}

uint64_t host_splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

}  // namespace
}  // namespace tufrg

using namespace tufrg;

struct tufrg_mlp {
  std::vector<int> widths;
  int nlayers = 0;
  int max_rows = 0, max_width = 0;
  int64_t nparams = 0;
  std::vector<int64_t> woff, boff;       // offsets of W_l and b_l in the flat vectors
  hipStream_t stream = nullptr;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // params, grads, Adam moments
  std::vector<float*> Z, A;              // per layer [max_rows][width_l], l = 1..L
  float *d0 = nullptr, *d1 = nullptr;    // delta ping-pong [max_rows][max_width]
  float *part = nullptr;                 // split-K partials
  int64_t part_cap = 0;
  float *xb = nullptr, *yb = nullptr;    // minibatch staging
  double *lpart = nullptr, *loss = nullptr;
  int64_t adam_t = 0;
  std::vector<void*> allocations;
  std::string err;
};

namespace {

thread_local std::string g_mlp_error;

tufrg_status mfail(tufrg_mlp* n, tufrg_status st, const std::string& msg) {
  if (n) n->err = msg;
  g_mlp_error = msg;
  return st;
}

#define MLP_TRY(net, expr)                                                                \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return mfail(net, TUFRG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)

template <class T>
tufrg_status malloc_dev(tufrg_mlp* n, size_t count, T** out) {
  void* ptr = nullptr;
  if (hipMalloc(&ptr, std::max<size_t>(count * sizeof(T), 16)) != hipSuccess)
    return mfail(n, TUFRG_ENOMEM, "hipMalloc failed (mlp)");
  n->allocations.push_back(ptr);
  *out = static_cast<T*>(ptr);
  return TUFRG_OK;
}

void gemm(hipStream_t s, int passes, const GemmArgs& a, int splits) {
  const dim3 grid((a.N + kTN - 1) / kTN, (a.M + kTM - 1) / kTM, splits);
  const bool vec = !a.transA && a.transB && a.lda % 4 == 0 && a.ldb % 4 == 0 &&
                   reinterpret_cast<uintptr_t>(a.A) % 16 == 0 && reinterpret_cast<uintptr_t>(a.B) % 16 == 0;
  if (passes == 3) {
    if (vec) hipLaunchKernelGGL((k_gemm<3, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_gemm<3, false>), grid, dim3(256), 0, s, a);
  } else {
    if (vec) hipLaunchKernelGGL((k_gemm<1, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_gemm<1, false>), grid, dim3(256), 0, s, a);
  }
}

GemmArgs base_args() {
  GemmArgs a;
  std::memset(&a, 0, sizeof a);
  return a;
}

// forward pass of `rows` rows of x on stream st; the last layer writes to
// out (ldc = nout)
void forward(tufrg_mlp* n, const float* x, int rows, float* out, bool keep_z, hipStream_t st) {
  const float* a_prev = x;
  for (int l = 0; l < n->nlayers; ++l) {
    const int in = n->widths[l], o = n->widths[l + 1];
    const bool last = l + 1 == n->nlayers;
    GemmArgs a = base_args();
    a.A = a_prev;
    a.lda = in;
    a.B = n->p + n->woff[l];
    a.ldb = in;
    a.transB = 1;
    a.C = last ? out : n->A[l];
    a.ldc = o;
    a.bias = n->p + n->boff[l];
    a.M = rows;
    a.N = o;
    a.K = in;
    a.kps = ((in + 31) / 32) * 32;
    a.epi = last ? kBias : kBiasSilu;
    a.Zs = (!last && keep_z) ? n->Z[l] : nullptr;
    a.ldz = o;
    gemm(st, 3, a, 1);
    a_prev = n->A[l];
  }
}

// loss and gradient of `rows` rows (x, y) into n->g; loss into n->loss[slot]
void forward_backward(tufrg_mlp* n, const float* x, const float* y, int rows, int slot) {
  const int L = n->nlayers, nout = n->widths[L];
  float* outL = n->A[L - 1];
  forward(n, x, rows, outL, true, n->stream);
  const int64_t ne = (int64_t)rows * nout;
  const int lblocks = (int)((ne + 255) / 256);
  float* delta = n->d0;
  float* other = n->d1;
  hipLaunchKernelGGL(k_loss, dim3(lblocks), dim3(256), 0, n->stream, outL, y, ne,
                     2.0f / (float)ne, delta, n->lpart);
  hipLaunchKernelGGL(k_sum_double, dim3(1), dim3(64), 0, n->stream, n->lpart, lblocks,
                     1.0 / (double)ne, n->loss + slot);
  for (int l = L - 1; l >= 0; --l) {
    const int in = n->widths[l], o = n->widths[l + 1];
    const float* a_prev = l == 0 ? x : n->A[l - 1];
    // dW_l = delta^T a_prev, split over rows, summed in split order
    const int kps = 256;
    const int splits = (rows + kps - 1) / kps;
    GemmArgs a = base_args();
    a.A = delta;
    a.lda = o;
    a.transA = 1;
    a.B = a_prev;
    a.ldb = in;
    a.C = n->part;
    a.ldc = in;
    a.split_stride = (int64_t)o * in;
    a.M = o;
    a.N = in;
    a.K = rows;
    a.kps = kps;
    a.epi = kStore;
    gemm(n->stream, 1, a, splits);
    const int64_t nw = (int64_t)o * in;
    hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, n->stream,
                       n->part, splits, a.split_stride, nw, n->g + n->woff[l]);
    // db_l = column sums of delta
    const int chunks = (rows + 255) / 256;
    hipLaunchKernelGGL(k_colsum_part, dim3((o + 255) / 256, chunks), dim3(256), 0, n->stream, delta,
                       rows, o, n->part);
    hipLaunchKernelGGL(k_sum_splits, dim3((o + 255) / 256), dim3(256), 0, n->stream, n->part, chunks,
                       (int64_t)o, (int64_t)o, n->g + n->boff[l]);
    if (l == 0) break;
    // delta_{l-1} = (delta W_l) * silu'(z_{l-1})
    GemmArgs b = base_args();
    b.A = delta;
    b.lda = o;
    b.B = n->p + n->woff[l];
    b.ldb = in;
    b.C = other;
    b.ldc = in;
    b.Zp = n->Z[l - 1];
    b.ldzp = in;
    b.M = rows;
    b.N = in;
    b.K = o;
    b.kps = ((o + 31) / 32) * 32;
    b.epi = kDsilu;
    gemm(n->stream, 1, b, 1);
    std::swap(delta, other);
  }
}

}  // namespace

namespace tufrg {

void mlp_forward_on(tufrg_mlp* n, const float* x, float* y, int64_t rows, hipStream_t s) {
  const int nin = n->widths[0], nout = n->widths[n->nlayers];
  for (int64_t r0 = 0; r0 < rows; r0 += n->max_rows) {
    const int r = (int)std::min<int64_t>(n->max_rows, rows - r0);
    forward(n, x + r0 * nin, r, y + r0 * nout, false, s);
  }
}

int mlp_width(const tufrg_mlp* n, int i) { return i < 0 ? n->widths[n->nlayers] : n->widths[i]; }

int mlp_max_rows(const tufrg_mlp* n) { return n->max_rows; }

}  // namespace tufrg

extern "C" {

tufrg_status tufrg_mlp_create(const int32_t* widths, int32_t nwidths, int32_t max_rows, uint64_t seed,
                              void* stream, tufrg_mlp** out) {
  if (!out) return mfail(nullptr, TUFRG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!widths || nwidths < 2) return mfail(nullptr, TUFRG_EINVAL, "need at least two widths");
  for (int i = 0; i < nwidths; ++i)
    if (widths[i] < 1 || widths[i] > 4096) return mfail(nullptr, TUFRG_EINVAL, "widths must be in 1..4096");
  if (max_rows < 1 || max_rows > (1 << 22)) return mfail(nullptr, TUFRG_EINVAL, "max_rows must be in 1..4194304");
  auto* n = new tufrg_mlp();
  n->widths.assign(widths, widths + nwidths);
  n->nlayers = nwidths - 1;
  n->max_rows = max_rows;
  n->max_width = *std::max_element(widths, widths + nwidths);
  n->stream = static_cast<hipStream_t>(stream);
  int64_t o = 0;
  for (int l = 0; l < n->nlayers; ++l) {
    n->woff.push_back(o);
    o += (int64_t)widths[l] * widths[l + 1];
    n->boff.push_back(o);
    o += widths[l + 1];
  }
  n->nparams = o;
  // Glorot-uniform weights from a counter-based generator, zero biases
  std::vector<float> init((size_t)o, 0.0f);
  for (int l = 0; l < n->nlayers; ++l) {
    const double lim = std::sqrt(6.0 / (double)(widths[l] + widths[l + 1]));
    const int64_t cnt = (int64_t)widths[l] * widths[l + 1];
    for (int64_t i = 0; i < cnt; ++i) {
      const uint64_t h = host_splitmix64(seed ^ host_splitmix64((uint64_t)(n->woff[l] + i)));
      const double u = (double)(h >> 11) * (1.0 / 9007199254740992.0);
      init[(size_t)(n->woff[l] + i)] = (float)((2.0 * u - 1.0) * lim);
    }
  }
  tufrg_status st = TUFRG_OK;
  auto bad = [&](tufrg_status s) {
    std::string m = n->err;
    tufrg_mlp_free(n);
    return mfail(nullptr, s, m);
  };
  if ((st = malloc_dev(n, (size_t)o, &n->p)) || (st = malloc_dev(n, (size_t)o, &n->g)) ||
      (st = malloc_dev(n, (size_t)o, &n->m)) || (st = malloc_dev(n, (size_t)o, &n->v)))
    return bad(st);
  n->Z.assign(n->nlayers, nullptr);
  n->A.assign(n->nlayers, nullptr);
  for (int l = 0; l < n->nlayers; ++l) {
    if ((st = malloc_dev(n, (size_t)max_rows * widths[l + 1], &n->Z[l])) ||
        (st = malloc_dev(n, (size_t)max_rows * widths[l + 1], &n->A[l])))
      return bad(st);
  }
  const size_t dsz = (size_t)max_rows * n->max_width;
  int64_t pc = 0;
  for (int l = 0; l < n->nlayers; ++l)
    pc = std::max<int64_t>(pc, (int64_t)((max_rows + 255) / 256) * widths[l] * widths[l + 1]);
  pc = std::max<int64_t>(pc, (int64_t)((max_rows + 255) / 256) * n->max_width);
  n->part_cap = pc;
  if ((st = malloc_dev(n, dsz, &n->d0)) || (st = malloc_dev(n, dsz, &n->d1)) ||
      (st = malloc_dev(n, (size_t)pc, &n->part)) ||
      (st = malloc_dev(n, (size_t)max_rows * widths[0], &n->xb)) ||
      (st = malloc_dev(n, (size_t)max_rows * widths[nwidths - 1], &n->yb)) ||
      (st = malloc_dev(n, (size_t)((int64_t)max_rows * widths[nwidths - 1] + 255) / 256 + 1, &n->lpart)) ||
      (st = malloc_dev(n, (size_t)1 << 20, &n->loss)))
    return bad(st);
  if (hipMemcpy(n->p, init.data(), sizeof(float) * o, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(n->m, 0, sizeof(float) * o) != hipSuccess || hipMemset(n->v, 0, sizeof(float) * o) != hipSuccess ||
      hipMemset(n->g, 0, sizeof(float) * o) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
    return bad(mfail(n, TUFRG_EHIP, "mlp initialisation copy failed"));
  *out = n;
  return TUFRG_OK;
}

tufrg_status tufrg_mlp_nparams(const tufrg_mlp* n, int64_t* count) {
  if (!n || !count) return mfail(nullptr, TUFRG_EINVAL, "NULL argument");
  *count = n->nparams;
  return TUFRG_OK;
}

tufrg_status tufrg_mlp_get_params(tufrg_mlp* n, float* dst) {
  if (!n || !dst) return mfail(n, TUFRG_EINVAL, "NULL argument");
  MLP_TRY(n, hipMemcpyAsync(dst, n->p, sizeof(float) * n->nparams, hipMemcpyDeviceToDevice, n->stream));
  return TUFRG_OK;
}

tufrg_status tufrg_mlp_set_params(tufrg_mlp* n, const float* src) {
  if (!n || !src) return mfail(n, TUFRG_EINVAL, "NULL argument");
  MLP_TRY(n, hipMemcpyAsync(n->p, src, sizeof(float) * n->nparams, hipMemcpyDeviceToDevice, n->stream));
  return TUFRG_OK;
}

tufrg_status tufrg_mlp_forward(tufrg_mlp* n, const float* x, float* y, int64_t rows) {
  if (!n || !x || !y) return mfail(n, TUFRG_EINVAL, "NULL argument");
  if (rows < 0) return mfail(n, TUFRG_EINVAL, "rows must be >= 0");
  const int nin = n->widths[0], nout = n->widths[n->nlayers];
  for (int64_t r0 = 0; r0 < rows; r0 += n->max_rows) {
    const int r = (int)std::min<int64_t>(n->max_rows, rows - r0);
    forward(n, x + r0 * nin, r, y + r0 * nout, false, n->stream);
  }
  MLP_TRY(n, hipGetLastError());
  return TUFRG_OK;
}

tufrg_status tufrg_mlp_gradient(tufrg_mlp* n, const float* x, const float* y, int64_t rows, float* grad,
                                double* loss) {
  if (!n || !x || !y) return mfail(n, TUFRG_EINVAL, "NULL argument");
  if (rows < 1 || rows > n->max_rows) return mfail(n, TUFRG_EINVAL, "rows must be in 1..max_rows");
  forward_backward(n, x, y, (int)rows, 0);
  if (grad)
    MLP_TRY(n, hipMemcpyAsync(grad, n->g, sizeof(float) * n->nparams, hipMemcpyDeviceToDevice, n->stream));
  if (loss) {
    MLP_TRY(n, hipMemcpyAsync(loss, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    MLP_TRY(n, hipStreamSynchronize(n->stream));
  }
  MLP_TRY(n, hipGetLastError());
  return TUFRG_OK;
}

tufrg_status tufrg_mlp_train(tufrg_mlp* n, const float* x, const float* y, int64_t rows, int32_t steps,
                             int32_t batch, float lr, uint64_t seed, double* loss_hist) {
  if (!n || !x || !y) return mfail(n, TUFRG_EINVAL, "NULL argument");
  if (rows < 1 || steps < 0 || batch < 1 || batch > n->max_rows || !(lr > 0.f))
    return mfail(n, TUFRG_EINVAL, "need rows >= 1, steps >= 0, 1 <= batch <= max_rows, lr > 0");
  if (loss_hist && steps > (1 << 20)) return mfail(n, TUFRG_EINVAL, "steps > 2^20 with a loss history");
  const int nin = n->widths[0], nout = n->widths[n->nlayers];
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int s = 0; s < steps; ++s) {
    hipLaunchKernelGGL(k_gather_rows, dim3(batch), dim3(64), 0, n->stream, x, nin, y, nout, rows, batch,
                       seed, (uint64_t)s, n->xb, n->yb);
    forward_backward(n, n->xb, n->yb, batch, loss_hist ? s : 0);
    // cosine decay of the learning rate to 1% over the call
    const double frac = steps > 1 ? (double)s / (double)(steps - 1) : 0.0;
    const float lr_s = (float)(lr * (0.01 + 0.99 * 0.5 * (1.0 + std::cos(M_PI * frac))));
    ++n->adam_t;
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)n->adam_t));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)n->adam_t));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n->nparams + 255) / 256)), dim3(256), 0, n->stream, n->p,
                       n->g, n->m, n->v, n->nparams, lr_s, b1, b2, eps, c1, c2);
  }
  if (loss_hist && steps > 0) {
    MLP_TRY(n, hipMemcpyAsync(loss_hist, n->loss, sizeof(double) * steps, hipMemcpyDeviceToHost, n->stream));
  }
  MLP_TRY(n, hipStreamSynchronize(n->stream));
  MLP_TRY(n, hipGetLastError());
  return TUFRG_OK;
}

void tufrg_mlp_free(tufrg_mlp* n) {
  if (!n) return;
  if (!n->allocations.empty()) (void)hipDeviceSynchronize();
  for (void* p : n->allocations) (void)hipFree(p);
  delete n;
}

const char* tufrg_mlp_last_error(const tufrg_mlp* n) {
  if (n) return n->err.c_str();
  return g_mlp_error.c_str();
}

}  // extern "C"
