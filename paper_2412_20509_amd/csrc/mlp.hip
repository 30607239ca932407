// Warm-start encoder: an MLP log(1 + y_i) -> 256 -> 256 -> d (GELU) trained
// with Adam in float32 and run for inference with bfloat16 operands, on the
// gfx950 matrix cores.
//
// gemm_kernel computes C = op(A) op(B) for row-major operands, with
//   * op = identity or transpose for each operand,
//   * an operand that is a matrix of int32 counts read as log(1 + y),
//   * fused epilogues: + bias, + bias then GELU (the pre-activation is kept for
//     the backward pass), or * GELU'(z) (backward through the activation),
// on 64 x 64 output tiles (4 wavefronts, 2 x 2 MFMA 16x16 tiles each), K in
// steps of 32 staged through LDS.  Tiles of one output row band are mapped to
// the same XCD (workgroups are dealt to the 8 XCDs round robin) so that they
// share the band's operand reads in one L2.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gmf.h"
#include "gmf_kernels.hpp"

namespace gmf {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

enum { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_BWD = 3 };
constexpr int TM = 64, TN = 64, TK = 32;

struct GemmArgs {
  const void* A; const void* B;
  int64_t lda, ldb;
  float* C; int64_t ldc;
  int M, N, K;
  const float* bias;   // N
  float* Zout;         // EPI_BIAS_GELU: pre-activation, leading dim ldc
  const float* Zin;    // EPI_GELU_BWD: pre-activation, leading dim ldc
  int mtiles, ntiles;
  int kchunk;          // K range of blockIdx.y: [y kchunk, (y+1) kchunk) (multiple of TK)
  int64_t cstride;     // output offset of blockIdx.y (split K writes partial products)
};

__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
  return cdf + z * pdf;
}

// Operand modes: 0 = float values, 1 = int32 counts read as log(1 + y),
// 2 = float32 counts read as log(1 + y).
template <int MODE>
__device__ __forceinline__ float load_elem(const void* p, int64_t idx) {
  if constexpr (MODE == 1) return log1pf((float)static_cast<const int*>(p)[idx]);
  else if constexpr (MODE == 2) return log1pf(static_cast<const float*>(p)[idx]);
  else return static_cast<const float*>(p)[idx];
}

template <int PREC, bool TA, bool TB, int A_COUNTS, int B_COUNTS, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  using TE = typename std::conditional<PREC == kF32, float, __bf16>::type;
  constexpr int PAD = (PREC == kF32) ? 4 : 8;
  __shared__ alignas(16) TE As[TM][TK + PAD];
  __shared__ alignas(16) TE Bs[TN][TK + PAD];
  // XCD-aware tile order: the ntiles tiles of one row band sit 8 ids apart
  const int b = blockIdx.x;
  const int group = b / (8 * g.ntiles);
  const int within = b % (8 * g.ntiles);
  const int mt = group * 8 + (within % 8);
  const int nt = within / 8;
  if (mt >= g.mtiles) return;
  const int m0 = mt * TM, n0 = nt * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, gq = lane >> 4;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  floatx4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int kb = blockIdx.y * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  float* const Cout = g.C + blockIdx.y * g.cstride;
  for (int k0 = kb; k0 < ke; k0 += TK) {
    __syncthreads();
    // A tile: element (m0+i, k0+kk) -> As[i][kk]
    if constexpr (!TA) {
      const int i = tid / 4, kk0 = (tid % 4) * 8;
      const int m = m0 + i;
      for (int u = 0; u < 8; ++u) {
        const int k = k0 + kk0 + u;
        const float v = (m < g.M && k < g.K) ? load_elem<A_COUNTS>(g.A, (int64_t)m * g.lda + k) : 0.f;
        As[i][kk0 + u] = (TE)v;
      }
    } else {
      const int kk = tid / 8, i0 = (tid % 8) * 8;
      const int k = k0 + kk;
      for (int u = 0; u < 8; ++u) {
        const int m = m0 + i0 + u;
        const float v = (m < g.M && k < g.K) ? load_elem<A_COUNTS>(g.A, (int64_t)k * g.lda + m) : 0.f;
        As[i0 + u][kk] = (TE)v;
      }
    }
    // B tile: element (k0+kk, n0+j) -> Bs[j][kk]
    if constexpr (!TB) {
      const int kk = tid / 8, j0 = (tid % 8) * 8;
      const int k = k0 + kk;
      for (int u = 0; u < 8; ++u) {
        const int n = n0 + j0 + u;
        const float v = (n < g.N && k < g.K) ? load_elem<B_COUNTS>(g.B, (int64_t)k * g.ldb + n) : 0.f;
        Bs[j0 + u][kk] = (TE)v;
      }
    } else {
      const int j = tid / 4, kk0 = (tid % 4) * 8;
      const int n = n0 + j;
      for (int u = 0; u < 8; ++u) {
        const int k = k0 + kk0 + u;
        const float v = (n < g.N && k < g.K) ? load_elem<B_COUNTS>(g.B, (int64_t)n * g.ldb + k) : 0.f;
        Bs[j][kk0 + u] = (TE)v;
      }
    }
    __syncthreads();
    if constexpr (PREC == kF32) {
      for (int ks = 0; ks < TK / 4; ++ks) {
        float a[2], bb[2];
        for (int i = 0; i < 2; ++i) a[i] = As[wm + 16 * i + l16][4 * ks + gq];
        for (int j = 0; j < 2; ++j) bb[j] = Bs[wn + 16 * j + l16][4 * ks + gq];
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bb[j], acc[i][j], 0, 0, 0);
      }
    } else {
      bf16x8 a[2], bb[2];
      for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * i + l16][8 * gq]);
      for (int j = 0; j < 2; ++j) bb[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * j + l16][8 * gq]);
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
  }
  // epilogue: lane holds rows 4gq+v of each 16x16 tile, column l16
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn + 16 * j + l16;
      if (n >= g.N) continue;
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + 16 * i + 4 * gq + v;
        if (m >= g.M) continue;
        float x = acc[i][j][v];
        const int64_t ci = (int64_t)m * g.ldc + n;
        if constexpr (EPI == EPI_BIAS) x += g.bias[n];
        if constexpr (EPI == EPI_BIAS_GELU) {
          x += g.bias[n];
          g.Zout[ci] = x;
          x = gelu_f(x);
        }
        if constexpr (EPI == EPI_GELU_BWD) x *= gelu_grad_f(g.Zin[ci]);
        Cout[ci] = x;
      }
    }
}

// Split-K epilogue: C = epilogue(sum over S partial products, in order).
template <int EPI>
__global__ void splitk_epilogue_kernel(const float* part, int S, int M, int N, const float* bias,
                                       float* C, int64_t ldc, float* Zout, const float* Zin) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)M * N) return;
  const int m = (int)(idx / N), n = (int)(idx % N);
  float x = 0.f;
  for (int s = 0; s < S; ++s) x += part[(int64_t)s * M * N + idx];
  const int64_t ci = (int64_t)m * ldc + n;
  if constexpr (EPI == EPI_BIAS) x += bias[n];
  if constexpr (EPI == EPI_BIAS_GELU) {
    x += bias[n];
    Zout[ci] = x;
    x = gelu_f(x);
  }
  if constexpr (EPI == EPI_GELU_BWD) x *= gelu_grad_f(Zin[ci]);
  C[ci] = x;
}

constexpr int kMaxSplit = 8;

// C = op(A) op(B) with the epilogue.  Float32 products with few output tiles
// and a long K (the first layer of a training batch) split K over up to
// kMaxSplit workgroups per tile when a buffer of kMaxSplit * M * N floats is
// given; bfloat16 products never split (their K order is fixed).
template <int PREC, bool TA, bool TB, int AC, int BC, int EPI>
hipError_t gemm(const GemmArgs& a0, hipStream_t s, float* split_buf = nullptr,
                int64_t split_cap = 0) {
  GemmArgs a = a0;
  a.mtiles = (a.M + TM - 1) / TM;
  a.ntiles = (a.N + TN - 1) / TN;
  const int groups = (a.mtiles + 7) / 8;
  const int grid = groups * 8 * a.ntiles;
  if (a.M <= 0 || a.N <= 0) return hipSuccess;
  int S = 1;
  if (PREC == kF32 && split_buf && a.mtiles * a.ntiles < 64 && a.K >= 1024 &&
      (int64_t)kMaxSplit * a.M * a.N <= split_cap)
    S = std::min(kMaxSplit, a.K / 256);
  if (S <= 1) {
    a.kchunk = (a.K + TK - 1) / TK * TK;
    a.cstride = 0;
    hipLaunchKernelGGL((gemm_kernel<PREC, TA, TB, AC, BC, EPI>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  GemmArgs p = a;
  p.kchunk = ((a.K + S - 1) / S + TK - 1) / TK * TK;
  S = (a.K + p.kchunk - 1) / p.kchunk;
  p.C = split_buf;
  p.ldc = a.N;
  p.cstride = (int64_t)a.M * a.N;
  hipLaunchKernelGGL((gemm_kernel<PREC, TA, TB, AC, BC, EPI_NONE>), dim3(grid, S), dim3(256), 0, s, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)a.M * a.N;
  hipLaunchKernelGGL((splitk_epilogue_kernel<EPI>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     split_buf, S, a.M, a.N, a.bias, a.C, a.ldc, a.Zout, a.Zin);
  return hipGetLastError();
}

// db[n] = sum_m D[m][n]: 64 columns per workgroup, rows split over 4 lanes
// groups (rows r = 4i + part), float64, then the four parts in order.
__global__ void colsum_kernel(const float* D, int M, int N, float* out) {
  __shared__ double red[4][64];
  const int t = threadIdx.x & 63, part = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + t;
  double s = 0.0;
  if (n < N)
    for (int m = part; m < M; m += 4) s += (double)D[(int64_t)m * N + n];
  red[part][t] = s;
  __syncthreads();
  if (part == 0 && n < N) out[n] = (float)(((red[0][t] + red[1][t]) + red[2][t]) + red[3][t]);
}

// dO = 2 (O - U) / (B d); loss partial sums of (O - U)^2 per block.
__global__ void mse_grad_kernel(const float* O, const float* U, int64_t count, float scale,
                                float* dO, double* partial) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) {
    const float r = O[i] - U[i];
    dO[i] = scale * r;
    acc += (double)r * r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Adam with bias correction and decoupled weight decay over a flat buffer.
__global__ void adam_kernel(float* p, const float* gr, float* m, float* v, int64_t count, float lr,
                            float b1, float b2, float eps, float wd, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const float g = gr[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps) - lr * wd * p[i];
}

__global__ void sum_kernel(const double* partial, int count, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < count; ++i) s += partial[i];
    *out = s;
  }
}

thread_local std::string g_err;
int efail(int code, const std::string& m) {
  g_err = m;
  return code;
}
#define EHIP(expr)                                                                \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) return ::gmf::efail(GMF_EDEVICE, std::string(#expr) + ": " + \
                                                        hipGetErrorString(e_));   \
  } while (0)

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct EncPlan {
  int m, H, d, batch;
  int64_t nparam;
  int64_t oW1, ob1, oW2, ob2, oW3, ob3;   // offsets (floats) inside the flat parameter vector
  size_t o_P, o_G, o_M, o_V, o_Z1, o_H1, o_Z2, o_H2, o_O, o_dO, o_dH, o_dZ, o_part, o_scal, total;
  int64_t inf_rows;   // rows per inference chunk
  // bfloat16 weights of the fused inference kernel (zero-padded): W1 H x k1p,
  // W2 H x H, W3 d3p x H with k1p = m rounded up to 32, d3p = d rounded up to 16
  int k1p, d3p;
  size_t o_W1b, o_W2b, o_W3b;
  size_t o_split;      // split-K partial products of a training batch's first layer
};

void plan_enc(const gmf_mlp_config* c, EncPlan& E) {
  E.m = c->m; E.H = c->hidden; E.d = c->d; E.batch = c->batch;
  int64_t o = 0;
  E.oW1 = o; o += (int64_t)E.H * E.m;
  E.ob1 = o; o += E.H;
  E.oW2 = o; o += (int64_t)E.H * E.H;
  E.ob2 = o; o += E.H;
  E.oW3 = o; o += (int64_t)E.d * E.H;
  E.ob3 = o; o += E.d;
  E.nparam = o;
  E.inf_rows = 65536;
  const int64_t rows = std::max<int64_t>(E.batch, E.inf_rows);
  size_t b = 0;
  auto take = [&](size_t bytes) { size_t at = b; b = al(b + bytes); return at; };
  E.o_P = take(4 * E.nparam);
  E.o_G = take(4 * E.nparam);
  E.o_M = take(4 * E.nparam);
  E.o_V = take(4 * E.nparam);
  E.o_Z1 = take(4 * rows * E.H);
  E.o_H1 = take(4 * rows * E.H);
  E.o_Z2 = take(4 * rows * E.H);
  E.o_H2 = take(4 * rows * E.H);
  E.o_O = take(4 * rows * E.d);
  E.o_dO = take(4 * (int64_t)E.batch * E.d);
  E.o_dH = take(4 * (int64_t)E.batch * E.H);
  E.o_dZ = take(4 * (int64_t)E.batch * E.H);
  E.o_part = take(8 * 256);
  E.o_scal = take(8 * 4);
  E.o_split = take(4 * (size_t)kMaxSplit * E.batch * E.H);
  E.k1p = (E.m + 31) / 32 * 32;
  E.d3p = (E.d + 15) / 16 * 16;
  E.o_W1b = take(2 * (size_t)E.H * E.k1p);
  E.o_W2b = take(2 * (size_t)E.H * E.H);
  E.o_W3b = take(2 * (size_t)E.d3p * E.H);
  E.total = b;
}

struct Enc {
  gmf_mlp_config cfg;
  EncPlan E;
  char* ws;
  hipStream_t st;
  int64_t t = 0;   // Adam updates done
  bool wb_valid = false;   // the bfloat16 weight copies match the weights
  template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  float* P(int64_t off) const { return at<float>(E.o_P) + off; }
  float* G(int64_t off) const { return at<float>(E.o_G) + off; }
};

GemmArgs gargs(const void* A, int64_t lda, const void* B, int64_t ldb, float* C, int64_t ldc, int M,
               int N, int K) {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc; g.M = M; g.N = N; g.K = K;
  return g;
}

// Forward of `rows` rows (Y counts, row stride m): Z1/H1/Z2/H2/O in the workspace.
template <int PREC, int COUNTS>
int forward(Enc* e, const void* Y, int rows) {
  const EncPlan& E = e->E;
  GemmArgs g = gargs(Y, E.m, e->P(E.oW1), E.m, e->at<float>(E.o_H1), E.H, rows, E.H, E.m);
  g.bias = e->P(E.ob1);
  g.Zout = e->at<float>(E.o_Z1);
  EHIP((gemm<PREC, false, true, COUNTS, false, EPI_BIAS_GELU>(
      g, e->st, e->at<float>(E.o_split), (int64_t)kMaxSplit * E.batch * E.H)));
  g = gargs(e->at<float>(E.o_H1), E.H, e->P(E.oW2), E.H, e->at<float>(E.o_H2), E.H, rows, E.H, E.H);
  g.bias = e->P(E.ob2);
  g.Zout = e->at<float>(E.o_Z2);
  EHIP((gemm<PREC, false, true, false, false, EPI_BIAS_GELU>(g, e->st)));
  g = gargs(e->at<float>(E.o_H2), E.H, e->P(E.oW3), E.H, e->at<float>(E.o_O), E.d, rows, E.d, E.H);
  g.bias = e->P(E.ob3);
  EHIP((gemm<PREC, false, true, false, false, EPI_BIAS>(g, e->st)));
  return GMF_OK;
}

// Loss partial and gradients (into the G buffer) of a batch of `rows` rows.
template <int COUNTS>
int grads_batch(Enc* e, const void* Y, const float* U, int rows, double* loss_partial) {
  const EncPlan& E = e->E;
  int rc = forward<kF32, COUNTS>(e, Y, rows);
  if (rc != GMF_OK) return rc;
  const int64_t cnt = (int64_t)rows * E.d;
  const float scale = 2.0f / (float)cnt;
  float* dO = e->at<float>(E.o_dO);
  hipLaunchKernelGGL(mse_grad_kernel, dim3(1), dim3(256), 0, e->st, e->at<float>(E.o_O), U, cnt,
                     scale, dO, loss_partial);
  EHIP(hipGetLastError());
  float* dH = e->at<float>(E.o_dH);
  float* dZ = e->at<float>(E.o_dZ);
  // layer 3: dW3 = dO' H2, db3 = colsum dO, dZ2 = (dO W3) * gelu'(Z2)
  EHIP((gemm<kF32, true, false, false, false, EPI_NONE>(
      gargs(dO, E.d, e->at<float>(E.o_H2), E.H, e->G(E.oW3), E.H, E.d, E.H, rows), e->st)));
  hipLaunchKernelGGL(colsum_kernel, dim3((E.d + 63) / 64), dim3(256), 0, e->st, dO, rows, E.d, e->G(E.ob3));
  GemmArgs g = gargs(dO, E.d, e->P(E.oW3), E.H, dZ, E.H, rows, E.H, E.d);
  g.Zin = e->at<float>(E.o_Z2);
  EHIP((gemm<kF32, false, false, false, false, EPI_GELU_BWD>(g, e->st)));
  // layer 2: dW2 = dZ2' H1, db2 = colsum dZ2, dZ1 = (dZ2 W2) * gelu'(Z1)
  EHIP((gemm<kF32, true, false, false, false, EPI_NONE>(
      gargs(dZ, E.H, e->at<float>(E.o_H1), E.H, e->G(E.oW2), E.H, E.H, E.H, rows), e->st)));
  hipLaunchKernelGGL(colsum_kernel, dim3((E.H + 63) / 64), dim3(256), 0, e->st, dZ, rows, E.H, e->G(E.ob2));
  g = gargs(dZ, E.H, e->P(E.oW2), E.H, dH, E.H, rows, E.H, E.H);
  g.Zin = e->at<float>(E.o_Z1);
  EHIP((gemm<kF32, false, false, false, false, EPI_GELU_BWD>(g, e->st)));
  // layer 1: dW1 = dZ1' log1p(Y), db1 = colsum dZ1
  EHIP((gemm<kF32, true, false, false, COUNTS, EPI_NONE>(
      gargs(dH, E.H, Y, E.m, e->G(E.oW1), E.m, E.H, E.m, rows), e->st)));
  hipLaunchKernelGGL(colsum_kernel, dim3((E.H + 63) / 64), dim3(256), 0, e->st, dH, rows, E.H, e->G(E.ob1));
  EHIP(hipGetLastError());
  return GMF_OK;
}

// ------------------------------------------------------ fused inference --
// out = MLP(log(1 + Y)) for 64 rows per workgroup, all three layers in one
// kernel with bfloat16 operands and float32 accumulation: the layer-1 count
// tile is staged through LDS (double-buffered, the next tile's loads in
// flight during the current tile's products); the activations of a layer
// stay in LDS as bfloat16 and feed the next layer; only the d outputs of a
// row are written.  Wavefront w computes hidden columns [H/4 w, H/4 (w+1)) of
// layers 1 and 2 (NJ = H/64 16-column tiles) and rows [16 w, 16 w + 16) of
// layer 3.  Products, their order and the rounding points (the log1p counts,
// the weights and each layer's GELU output rounded to bfloat16) are those of
// the layer-by-layer path, so the results agree with it bit for bit.
struct FusedArgs {
  const void* Y;
  int64_t rows;
  int m, H, d, k1p, d3p;
  const __bf16* W1b; const float* b1;
  const __bf16* W2b; const float* b2;
  const __bf16* W3b; const float* b3;
  float* out;
};

constexpr int kFusedRows = 64;

template <int COUNTS, int NJ>
__global__ __launch_bounds__(256) void fused_forward_kernel(FusedArgs a) {
  constexpr int BM = kFusedRows;
  constexpr int HMAX = 64 * NJ;
  __shared__ alignas(16) __bf16 sA[2][BM][32 + 8];
  __shared__ alignas(16) __bf16 sH[BM][HMAX + 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * BM;
  const int colw = wave * 16 * NJ;
  floatx4 acc[4][NJ];
  // ---- layer 1: K = m in tiles of 32, counts staged through LDS
  const int sr = tid >> 2, sk = (tid & 3) * 8;   // this thread's staging slot
  const int64_t srow = row0 + sr;
  auto load_counts = [&](int k0, float (&v)[8]) {
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + sk + u;
      v[u] = (srow < a.rows && k < a.m) ? load_elem<COUNTS>(a.Y, srow * a.m + k) : 0.f;
    }
  };
  auto store_counts = [&](int buf, const float (&v)[8]) {
    const floatx8 x = {v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
    *reinterpret_cast<bf16x8*>(&sA[buf][sr][sk]) = __builtin_convertvector(x, bf16x8);
  };
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < NJ; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  float pre[8];
  load_counts(0, pre);
  store_counts(0, pre);
  __syncthreads();
  const int nk = a.k1p / 32;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1, k0 = kt * 32;
    if (kt + 1 < nk) load_counts(k0 + 32, pre);
    bf16x8 av[4], bv[NJ];
    for (int i = 0; i < 4; ++i) av[i] = *reinterpret_cast<const bf16x8*>(&sA[buf][16 * i + l16][8 * g]);
    for (int j = 0; j < NJ; ++j)
      bv[j] = *reinterpret_cast<const bf16x8*>(a.W1b + (int64_t)(colw + 16 * j + l16) * a.k1p + k0 + 8 * g);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < NJ; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    if (kt + 1 < nk) store_counts(buf ^ 1, pre);
    __syncthreads();
  }
  // bias + GELU, bfloat16 into sH
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < NJ; ++j) {
      const int col = colw + 16 * j + l16;
      const float bb = a.b1[col];
      for (int v = 0; v < 4; ++v) sH[16 * i + 4 * g + v][col] = (__bf16)gelu_f(acc[i][j][v] + bb);
    }
  __syncthreads();
  // ---- layer 2: K = H from sH
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < NJ; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < a.H; k0 += 32) {
    bf16x8 av[4], bv[NJ];
    for (int i = 0; i < 4; ++i) av[i] = *reinterpret_cast<const bf16x8*>(&sH[16 * i + l16][k0 + 8 * g]);
    for (int j = 0; j < NJ; ++j)
      bv[j] = *reinterpret_cast<const bf16x8*>(a.W2b + (int64_t)(colw + 16 * j + l16) * a.H + k0 + 8 * g);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < NJ; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
  }
  __syncthreads();   // every wavefront has read layer 1's activations
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < NJ; ++j) {
      const int col = colw + 16 * j + l16;
      const float bb = a.b2[col];
      for (int v = 0; v < 4; ++v) sH[16 * i + 4 * g + v][col] = (__bf16)gelu_f(acc[i][j][v] + bb);
    }
  __syncthreads();
  // ---- layer 3: rows [16 wave, +16), d outputs in tiles of 16
  const int nj3 = a.d3p / 16;
  for (int j = 0; j < nj3; ++j) {
    floatx4 o = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < a.H; k0 += 32) {
      const bf16x8 av = *reinterpret_cast<const bf16x8*>(&sH[16 * wave + l16][k0 + 8 * g]);
      const bf16x8 bv = *reinterpret_cast<const bf16x8*>(a.W3b + (int64_t)(16 * j + l16) * a.H + k0 + 8 * g);
      o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, o, 0, 0, 0);
    }
    const int col = 16 * j + l16;
    if (col < a.d)
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + 16 * wave + 4 * g + v;
        if (row < a.rows) a.out[row * a.d + col] = o[v] + a.b3[col];
      }
  }
}

// float weights (rows x cols) -> bfloat16 (out_rows x out_cols, zero padded)
__global__ void weight_bf16_kernel(const float* W, int rows, int cols, __bf16* out, int out_rows,
                                   int out_cols) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)out_rows * out_cols) return;
  const int r = (int)(idx / out_cols), c = (int)(idx % out_cols);
  out[idx] = (r < rows && c < cols) ? (__bf16)W[(int64_t)r * cols + c] : (__bf16)0.f;
}

bool fused_supported(const EncPlan& E) { return E.H % 64 == 0 && E.H <= 256 && E.d <= 64; }

int refresh_bf16_weights(Enc* e) {
  const EncPlan& E = e->E;
  if (e->wb_valid) return GMF_OK;
  struct Job { int64_t src; int rows, cols; size_t dst; int orows, ocols; };
  const Job jobs[3] = {{E.oW1, E.H, E.m, E.o_W1b, E.H, E.k1p},
                       {E.oW2, E.H, E.H, E.o_W2b, E.H, E.H},
                       {E.oW3, E.d, E.H, E.o_W3b, E.d3p, E.H}};
  for (const Job& jb : jobs) {
    const int64_t n = (int64_t)jb.orows * jb.ocols;
    hipLaunchKernelGGL(weight_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, e->st,
                       e->P(jb.src), jb.rows, jb.cols, e->at<__bf16>(jb.dst), jb.orows, jb.ocols);
    EHIP(hipGetLastError());
  }
  e->wb_valid = true;
  return GMF_OK;
}

template <int COUNTS>
int fused_forward(Enc* e, const void* Y, int64_t rows, float* out) {
  const EncPlan& E = e->E;
  int rc = refresh_bf16_weights(e);
  if (rc != GMF_OK) return rc;
  FusedArgs f;
  f.Y = Y; f.rows = rows; f.m = E.m; f.H = E.H; f.d = E.d; f.k1p = E.k1p; f.d3p = E.d3p;
  f.W1b = e->at<__bf16>(E.o_W1b); f.b1 = e->P(E.ob1);
  f.W2b = e->at<__bf16>(E.o_W2b); f.b2 = e->P(E.ob2);
  f.W3b = e->at<__bf16>(E.o_W3b); f.b3 = e->P(E.ob3);
  f.out = out;
  const dim3 grid((unsigned)((rows + kFusedRows - 1) / kFusedRows));
  switch (E.H / 64) {
    case 1: hipLaunchKernelGGL((fused_forward_kernel<COUNTS, 1>), grid, dim3(256), 0, e->st, f); break;
    case 2: hipLaunchKernelGGL((fused_forward_kernel<COUNTS, 2>), grid, dim3(256), 0, e->st, f); break;
    case 3: hipLaunchKernelGGL((fused_forward_kernel<COUNTS, 3>), grid, dim3(256), 0, e->st, f); break;
    default: hipLaunchKernelGGL((fused_forward_kernel<COUNTS, 4>), grid, dim3(256), 0, e->st, f); break;
  }
  EHIP(hipGetLastError());
  return GMF_OK;
}

// One Adam step on the batch of `rows` rows.
template <int COUNTS>
int train_batch(Enc* e, const void* Y, const float* U, int rows, double* loss_partial) {
  const EncPlan& E = e->E;
  int rc = grads_batch<COUNTS>(e, Y, U, rows, loss_partial);
  if (rc != GMF_OK) return rc;
  e->t += 1;
  e->wb_valid = false;
  const gmf_mlp_config& c = e->cfg;
  const float c1 = (float)(1.0 - std::pow(c.beta1, (double)e->t));
  const float c2 = (float)(1.0 - std::pow(c.beta2, (double)e->t));
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((E.nparam + 255) / 256)), dim3(256), 0, e->st,
                     e->at<float>(E.o_P), e->at<float>(E.o_G), e->at<float>(E.o_M), e->at<float>(E.o_V),
                     E.nparam, (float)c.lr, (float)c.beta1, (float)c.beta2, (float)c.eps,
                     (float)c.weight_decay, c1, c2);
  EHIP(hipGetLastError());
  return GMF_OK;
}

}  // namespace
}  // namespace gmf

using gmf::Enc;
using gmf::EncPlan;

extern "C" {

void gmf_mlp_config_default(gmf_mlp_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->m = 1; c->hidden = 256; c->d = 1; c->batch = 256;
  c->lr = 1e-3; c->beta1 = 0.9; c->beta2 = 0.999; c->eps = 1e-8; c->weight_decay = 0.0;
}

size_t gmf_encoder_workspace_bytes(const gmf_mlp_config* c) {
  if (!c || c->m < 1 || c->hidden < 1 || c->d < 1 || c->batch < 1) return 0;
  EncPlan E;
  gmf::plan_enc(c, E);
  return E.total;
}

const char* gmf_encoder_last_error(void) { return gmf::g_err.c_str(); }

int gmf_encoder_init(void** enc_out, const gmf_mlp_config* c, void* ws, size_t ws_bytes,
                     void* stream, const float* W1, const float* b1, const float* W2,
                     const float* b2, const float* W3, const float* b3) {
  if (!enc_out || !c) return gmf::efail(GMF_EINVAL, "NULL argument");
  *enc_out = nullptr;
  if (c->m < 1 || c->hidden < 1 || c->d < 1 || c->batch < 1 || !(c->lr > 0))
    return gmf::efail(GMF_EINVAL, "bad encoder configuration");
  if (!W1 || !b1 || !W2 || !b2 || !W3 || !b3) return gmf::efail(GMF_EINVAL, "missing weights");
  EncPlan E;
  gmf::plan_enc(c, E);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) || ws_bytes < E.total)
    return gmf::efail(GMF_EWORKSPACE, "encoder workspace NULL, misaligned or too small");
  Enc* e = new Enc();
  e->cfg = *c;
  e->E = E;
  e->ws = static_cast<char*>(ws);
  e->st = static_cast<hipStream_t>(stream);
  const float* src[6] = {W1, b1, W2, b2, W3, b3};
  const int64_t off[6] = {E.oW1, E.ob1, E.oW2, E.ob2, E.oW3, E.ob3};
  const int64_t len[6] = {(int64_t)E.H * E.m, E.H, (int64_t)E.H * E.H, E.H, (int64_t)E.d * E.H, E.d};
  hipError_t err = hipSuccess;
  for (int i = 0; i < 6 && err == hipSuccess; ++i)
    err = hipMemcpyAsync(e->P(off[i]), src[i], 4 * len[i], hipMemcpyDeviceToDevice, e->st);
  if (err == hipSuccess) err = hipMemsetAsync(e->at<float>(E.o_M), 0, 4 * E.nparam, e->st);
  if (err == hipSuccess) err = hipMemsetAsync(e->at<float>(E.o_V), 0, 4 * E.nparam, e->st);
  if (err == hipSuccess) err = hipStreamSynchronize(e->st);
  if (err != hipSuccess) {
    delete e;
    return gmf::efail(GMF_EDEVICE, hipGetErrorString(err));
  }
  *enc_out = e;
  return GMF_OK;
}

int gmf_encoder_train(void* enc, const void* Y, int32_t y_dtype, const float* U, int64_t nrows,
                      int32_t epochs, double* loss_trace_host) {
  if (!enc || !Y || !U) return gmf::efail(GMF_EINVAL, "NULL argument");
  if (y_dtype != GMF_Y_INT32 && y_dtype != GMF_Y_FLOAT32) return gmf::efail(GMF_EINVAL, "bad y_dtype");
  Enc* e = static_cast<Enc*>(enc);
  const EncPlan& E = e->E;
  if (nrows < 1 || epochs < 0) return gmf::efail(GMF_EINVAL, "bad nrows/epochs");
  double* part = e->at<double>(E.o_part);
  double* scal = e->at<double>(E.o_scal);
  const int nb = (int)((nrows + E.batch - 1) / E.batch);
  for (int ep = 0; ep < epochs; ++ep) {
    for (int b = 0; b < nb; ++b) {
      const int64_t r0 = (int64_t)b * E.batch;
      const int rows = (int)std::min<int64_t>(E.batch, nrows - r0);
      const void* Yb = (y_dtype == GMF_Y_INT32)
                           ? static_cast<const void*>(static_cast<const int*>(Y) + r0 * E.m)
                           : static_cast<const void*>(static_cast<const float*>(Y) + r0 * E.m);
      int rc = (y_dtype == GMF_Y_INT32)
                   ? gmf::train_batch<1>(e, Yb, U + r0 * E.d, rows, part + (b % 256))
                   : gmf::train_batch<2>(e, Yb, U + r0 * E.d, rows, part + (b % 256));
      if (rc != GMF_OK) return rc;
      if (loss_trace_host && (b % 256 == 255 || b == nb - 1)) {
        // flush the batch losses of this window into the epoch total
        hipLaunchKernelGGL(gmf::sum_kernel, dim3(1), dim3(64), 0, e->st, part, (b % 256) + 1, scal);
        double s = 0;
        EHIP(hipMemcpyAsync(&s, scal, sizeof(double), hipMemcpyDeviceToHost, e->st));
        EHIP(hipStreamSynchronize(e->st));
        if (b < 256) loss_trace_host[ep] = 0;
        loss_trace_host[ep] += s;
      }
    }
    if (loss_trace_host) loss_trace_host[ep] /= (double)nrows * E.d;
  }
  EHIP(hipGetLastError());
  return GMF_OK;
}

int gmf_encoder_forward(void* enc, const void* Y, int32_t y_dtype, int64_t nrows, float* U_out,
                        int32_t bf16) {
  if (!enc || !Y || !U_out) return gmf::efail(GMF_EINVAL, "NULL argument");
  if (y_dtype != GMF_Y_INT32 && y_dtype != GMF_Y_FLOAT32) return gmf::efail(GMF_EINVAL, "bad y_dtype");
  Enc* e = static_cast<Enc*>(enc);
  const EncPlan& E = e->E;
  if (bf16 < 0 || bf16 > 2) return gmf::efail(GMF_EINVAL, "bf16 must be 0, 1 or 2");
  if (bf16 == 1 && gmf::fused_supported(E))
    return (y_dtype == GMF_Y_INT32) ? gmf::fused_forward<1>(e, Y, nrows, U_out)
                                    : gmf::fused_forward<2>(e, Y, nrows, U_out);
  for (int64_t r0 = 0; r0 < nrows; r0 += E.inf_rows) {
    const int rows = (int)std::min<int64_t>(E.inf_rows, nrows - r0);
    const void* Yb = (y_dtype == GMF_Y_INT32)
                         ? static_cast<const void*>(static_cast<const int*>(Y) + r0 * E.m)
                         : static_cast<const void*>(static_cast<const float*>(Y) + r0 * E.m);
    int rc;
    if (bf16) rc = (y_dtype == GMF_Y_INT32) ? gmf::forward<gmf::kBF16, 1>(e, Yb, rows)
                                           : gmf::forward<gmf::kBF16, 2>(e, Yb, rows);
    else rc = (y_dtype == GMF_Y_INT32) ? gmf::forward<gmf::kF32, 1>(e, Yb, rows)
                                      : gmf::forward<gmf::kF32, 2>(e, Yb, rows);
    if (rc != GMF_OK) return rc;
    EHIP(hipMemcpyAsync(U_out + r0 * E.d, e->at<float>(E.o_O), 4 * (int64_t)rows * E.d,
                        hipMemcpyDeviceToDevice, e->st));
  }
  return GMF_OK;
}

int gmf_encoder_get_weights(void* enc, float* W1, float* b1, float* W2, float* b2, float* W3,
                            float* b3) {
  if (!enc) return gmf::efail(GMF_EINVAL, "NULL argument");
  Enc* e = static_cast<Enc*>(enc);
  const EncPlan& E = e->E;
  float* dst[6] = {W1, b1, W2, b2, W3, b3};
  const int64_t off[6] = {E.oW1, E.ob1, E.oW2, E.ob2, E.oW3, E.ob3};
  const int64_t len[6] = {(int64_t)E.H * E.m, E.H, (int64_t)E.H * E.H, E.H, (int64_t)E.d * E.H, E.d};
  for (int i = 0; i < 6; ++i)
    if (dst[i]) EHIP(hipMemcpyAsync(dst[i], e->P(off[i]), 4 * len[i], hipMemcpyDeviceToDevice, e->st));
  EHIP(hipStreamSynchronize(e->st));
  return GMF_OK;
}

int gmf_encoder_loss_grad(void* enc, const void* Y, int32_t y_dtype, const float* U, int64_t nrows,
                          double* loss_host, float* grad_out) {
  if (!enc || !Y || !U) return gmf::efail(GMF_EINVAL, "NULL argument");
  Enc* e = static_cast<Enc*>(enc);
  const EncPlan& E = e->E;
  if (nrows < 1 || nrows > E.batch) return gmf::efail(GMF_EINVAL, "nrows must be in 1..batch");
  if (y_dtype != GMF_Y_INT32 && y_dtype != GMF_Y_FLOAT32) return gmf::efail(GMF_EINVAL, "bad y_dtype");
  double* part = e->at<double>(E.o_part);
  const int rc = (y_dtype == GMF_Y_INT32) ? gmf::grads_batch<1>(e, Y, U, (int)nrows, part)
                                          : gmf::grads_batch<2>(e, Y, U, (int)nrows, part);
  if (rc != GMF_OK) return rc;
  if (grad_out)
    EHIP(hipMemcpyAsync(grad_out, e->at<float>(E.o_G), 4 * E.nparam, hipMemcpyDeviceToDevice, e->st));
  double s = 0;
  EHIP(hipMemcpyAsync(&s, part, sizeof(double), hipMemcpyDeviceToHost, e->st));
  EHIP(hipStreamSynchronize(e->st));
  if (loss_host) *loss_host = s / ((double)nrows * E.d);
  return GMF_OK;
}

void gmf_encoder_destroy(void* enc) { delete static_cast<Enc*>(enc); }

}  // extern "C"
