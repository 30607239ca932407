// Identifiability post-processing in float64 on the device (Algorithm 2,
// constraints (A) then (B1)).
//
// (A): with D_G = (X'X)^-1 X'Gamma, D_U = (X'X)^-1 X'U, D_V = (Z'Z)^-1 Z'V
//      (all read off the Gram matrices of the two panels),
//        Gamma <- Gamma - X D_G + U' D_V',  U' = U - X D_U,
//        B     <- B + Z D_G' + V D_U',      V' = V - Z D_V.
//      Every new row is a fixed linear map of its old panel row, so the maps
//      are formed once (k x k matrices) and applied in one pass.
// (B1): U' V'^T = Q_u R_u R_v' Q_v' with R from CholeskyQR2 (Gram, Cholesky,
//      Gram of U' R1^-1, Cholesky again: R = R2 R1); the d x d core
//      C = R_u R_v' is split by a one-sided Jacobi SVD C = P S Q' (singular
//      values sorted decreasing), and U <- U' R_u^-1 P S, V <- V' R_v^-1 Q, which
//      equals the SVD route of Algorithm 2 without forming the n x m product.
//      Sign rule: the first non-zero entry (original order) of each V column
//      is made positive.
#include <hip/hip_runtime.h>

#include "gmf_kernels.hpp"

namespace gmf {

namespace {

constexpr int KM = 64;                    // leading dimension of small matrices
constexpr int SLOT = KM * KM;
constexpr int kGramBlocks = 128;
enum Slot { sGr = 0, sGc, sMr, sMc, sT1u, sT1v, sR1u, sR1v, sG2u, sG2v, sFu, sFv, sW0, sW1,
            sW2, sStatus, kSlots };

// Gram of rows: out[blk] = sum over its rows of y y', y = P_i[0:k] (T == null)
// or y = P_i[0:k] T (k x dt).  Fixed row order per block.
__global__ __launch_bounds__(256) void gram_kernel(const float* P, int KP, int64_t rows, int k,
                                                   const double* T, int dt, double* partial) {
  __shared__ double sy[32][KM + 1];
  const int dim = T ? dt : k;
  const int64_t chunk = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = min(rows, r0 + chunk);
  double acc[16];
  for (int e = 0; e < 16; ++e) acc[e] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += 32) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < 32 * KM; idx += 256) {
      const int rr = idx / KM, c = idx % KM;
      const int64_t row = rb + rr;
      double y = 0.0;
      if (row < r1 && c < dim) {
        if (!T) {
          y = (double)P[row * KP + c];
        } else {
          for (int a = 0; a < k; ++a) y += (double)P[row * KP + a] * T[a * KM + c];
        }
      }
      sy[rr][c] = y;
    }
    __syncthreads();
    const int nr = (int)min<int64_t>(32, r1 - rb);
    for (int e = 0; e < 16; ++e) {
      const int idx = threadIdx.x + 256 * e;
      const int a = idx / KM, b = idx % KM;
      if (a < dim && b < dim) {
        double s = 0.0;
        for (int rr = 0; rr < nr; ++rr) s += sy[rr][a] * sy[rr][b];
        acc[e] += s;
      }
    }
  }
  for (int e = 0; e < 16; ++e) partial[(int64_t)blockIdx.x * SLOT + threadIdx.x + 256 * e] = acc[e];
}

__global__ void sum_slots_kernel(const double* partial, int nblk, double* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= SLOT) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * SLOT + idx];
  out[idx] = s;
}

// ---- single-wavefront small dense linear algebra (lane = column index) ----
// Upper Cholesky A = R'R of the leading n x n block; returns false if not SPD.
__device__ bool chol_upper(const double* A, double* Rm, int n) {
  const int lane = threadIdx.x;
  for (int idx = lane; idx < SLOT; idx += 64) Rm[idx] = 0.0;
  __syncthreads();
  bool ok = true;
  for (int j = 0; j < n; ++j) {
    // R[j][j] = sqrt(A[j][j] - sum_{i<j} R[i][j]^2)
    double s = A[j * KM + j];
    for (int i = 0; i < j; ++i) s -= Rm[i * KM + j] * Rm[i * KM + j];
    if (!(s > 0.0)) ok = false;
    const double rjj = sqrt(fmax(s, 0.0));
    // R[j][c] = (A[j][c] - sum_{i<j} R[i][j] R[i][c]) / R[j][j], c > j
    const int c = lane;
    double v = 0.0;
    if (c > j && c < n) {
      v = A[j * KM + c];
      for (int i = 0; i < j; ++i) v -= Rm[i * KM + j] * Rm[i * KM + c];
      v /= rjj;
    }
    __syncthreads();
    if (c > j && c < n) Rm[j * KM + c] = v;
    if (lane == 0) Rm[j * KM + j] = rjj;
    __syncthreads();
  }
  return ok;
}

// X <- X R^-1 for an upper-triangular R (n x n), X has `rows` rows.
__device__ void right_solve_upper(double* X, int rows, const double* Rm, int n) {
  const int lane = threadIdx.x;
  for (int r = lane; r < rows; r += 64) {
    for (int j = 0; j < n; ++j) {
      double v = X[r * KM + j];
      for (int i = 0; i < j; ++i) v -= X[r * KM + i] * Rm[i * KM + j];
      X[r * KM + j] = v / Rm[j * KM + j];
    }
  }
  __syncthreads();
}

// C = A (ra x ka) * B (ka x cb); all with leading dimension KM.
__device__ void matmul(const double* A, const double* B, double* C, int ra, int ka, int cb) {
  for (int idx = threadIdx.x; idx < ra * cb; idx += 64) {
    const int i = idx / cb, j = idx % cb;
    double s = 0.0;
    for (int t = 0; t < ka; ++t) s += A[i * KM + t] * B[t * KM + j];
    C[i * KM + j] = s;
  }
  __syncthreads();
}

// Solve (A) X = Bm for SPD A (n x n, Cholesky) with `nc` right-hand columns.
__device__ bool spd_solve(const double* A, const double* Bm, double* X, int n, int nc,
                          double* work) {
  const bool ok = chol_upper(A, work, n);
  // R'R X = Bm: forward with R' then backward with R, one column per lane.
  const int c = threadIdx.x;
  if (c < nc) {
    for (int i = 0; i < n; ++i) {
      double v = Bm[i * KM + c];
      for (int t = 0; t < i; ++t) v -= work[t * KM + i] * X[t * KM + c];
      X[i * KM + c] = v / work[i * KM + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double v = X[i * KM + c];
      for (int t = i + 1; t < n; ++t) v -= work[i * KM + t] * X[t * KM + c];
      X[i * KM + c] = v / work[i * KM + i];
    }
  }
  __syncthreads();
  return ok;
}

__device__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One-sided Jacobi SVD of the d x d matrix in C (overwritten): on return
// C = P S (columns scaled), Vj holds Q, sig the singular values (unsorted).
__device__ void jacobi_svd(double* C, double* Vj, double* sig, int d) {
  const int lane = threadIdx.x;   // row index
  for (int idx = lane; idx < SLOT; idx += 64) Vj[idx] = ((idx / KM) == (idx % KM)) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off_max = 0.0;
    for (int i = 0; i < d - 1; ++i)
      for (int j = i + 1; j < d; ++j) {
        const double ci = lane < d ? C[lane * KM + i] : 0.0;
        const double cj = lane < d ? C[lane * KM + j] : 0.0;
        const double al = wave_sum(ci * ci);
        const double be = wave_sum(cj * cj);
        const double ga = wave_sum(ci * cj);
        const double scale = sqrt(al * be);
        if (scale == 0.0 || fabs(ga) <= 1e-17 * scale) continue;
        off_max = fmax(off_max, fabs(ga) / scale);
        const double zeta = (be - al) / (2.0 * ga);
        const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tt * tt);
        const double sn = cs * tt;
        if (lane < d) {
          C[lane * KM + i] = cs * ci - sn * cj;
          C[lane * KM + j] = sn * ci + cs * cj;
          const double vi = Vj[lane * KM + i], vj = Vj[lane * KM + j];
          Vj[lane * KM + i] = cs * vi - sn * vj;
          Vj[lane * KM + j] = sn * vi + cs * vj;
        }
        __syncthreads();
      }
    if (off_max < 1e-15) break;
  }
  for (int c = 0; c < d; ++c) {
    const double x = lane < d ? C[lane * KM + c] : 0.0;
    const double nrm = sqrt(wave_sum(x * x));
    if (lane == 0) sig[c] = nrm;
  }
  __syncthreads();
}

// Step 1: covariate maps (A) and the first Cholesky factors.
__global__ __launch_bounds__(64) void solve1_kernel(double* sm, int p, int q, int d) {
  const int k = p + q + d;
  const int lane = threadIdx.x;
  double* Gr = sm + sGr * SLOT;
  double* Gc = sm + sGc * SLOT;
  double* Mr = sm + sMr * SLOT;   // k x (q+d): rows [x | gamma | u] -> cols [gamma' | u']
  double* Mc = sm + sMc * SLOT;   // k x (p+d): rows [b | z | v] -> cols [b' | v']
  double* W0 = sm + sW0 * SLOT;
  double* W1 = sm + sW1 * SLOT;
  double* W2 = sm + sW2 * SLOT;
  double* status = sm + sStatus * SLOT;
  bool ok = true;
  // D_G (p x q) and D_U (p x d): (X'X) [D_G | D_U] = [X'Gamma | X'U]
  // right-hand sides: Gr[0:p, p:k]
  for (int idx = lane; idx < SLOT; idx += 64) { W0[idx] = 0.0; W1[idx] = 0.0; }
  __syncthreads();
  double* DGU = W1;   // p x (q+d)
  if (p > 0) {
    for (int idx = lane; idx < p * (q + d); idx += 64) {
      const int i = idx / (q + d), c = idx % (q + d);
      W0[i * KM + c] = Gr[i * KM + p + c];
    }
    __syncthreads();
    ok = spd_solve(Gr, W0, DGU, p, q + d, W2) && ok;
  }
  double* DV = sm + sT1v * SLOT;   // q x d, temporary (overwritten below)
  for (int idx = lane; idx < SLOT; idx += 64) { W0[idx] = 0.0; DV[idx] = 0.0; }
  __syncthreads();
  if (q > 0) {
    // (Z'Z) D_V = Z'V: Gc[p:p+q, p:p+q], rhs Gc[p:p+q, p+q:k]
    double* ZZ = sm + sR1v * SLOT;
    for (int idx = lane; idx < SLOT; idx += 64) ZZ[idx] = 0.0;
    __syncthreads();
    for (int idx = lane; idx < q * q; idx += 64) {
      const int i = idx / q, j = idx % q;
      ZZ[i * KM + j] = Gc[(p + i) * KM + p + j];
    }
    for (int idx = lane; idx < q * d; idx += 64) {
      const int i = idx / d, c = idx % d;
      W0[i * KM + c] = Gc[(p + i) * KM + p + q + c];
    }
    __syncthreads();
    ok = spd_solve(ZZ, W0, DV, q, d, W2) && ok;
  }
  // Row map Mr.
  for (int idx = lane; idx < SLOT; idx += 64) { Mr[idx] = 0.0; Mc[idx] = 0.0; }
  __syncthreads();
  for (int idx = lane; idx < k * (q + d); idx += 64) {
    const int a = idx / (q + d), c = idx % (q + d);
    double v = 0.0;
    if (c < q) {            // gamma'_c
      if (a < p) {          // -D_G[a][c] - sum_t D_U[a][t] D_V[c][t]
        v = -DGU[a * KM + c];
        for (int t = 0; t < d; ++t) v -= DGU[a * KM + q + t] * DV[c * KM + t];
      } else if (a < p + q) {
        v = (a - p == c) ? 1.0 : 0.0;
      } else {
        v = DV[c * KM + (a - p - q)];
      }
    } else {                // u'_{c-q}
      const int cc = c - q;
      if (a < p) v = -DGU[a * KM + q + cc];
      else if (a < p + q) v = 0.0;
      else v = (a - p - q == cc) ? 1.0 : 0.0;
    }
    Mr[a * KM + c] = v;
  }
  for (int idx = lane; idx < k * (p + d); idx += 64) {
    const int a = idx / (p + d), c = idx % (p + d);
    double v = 0.0;
    if (c < p) {            // b'_c = b + z D_G' + v D_U'
      if (a < p) v = (a == c) ? 1.0 : 0.0;
      else if (a < p + q) v = DGU[c * KM + (a - p)];
      else v = DGU[c * KM + q + (a - p - q)];
    } else {                // v'_{c-p} = v - z D_V
      const int cc = c - p;
      if (a < p) v = 0.0;
      else if (a < p + q) v = -DV[(a - p) * KM + cc];
      else v = (a - p - q == cc) ? 1.0 : 0.0;
    }
    Mc[a * KM + c] = v;
  }
  __syncthreads();
  // U'U' = Mu' Gr Mu with Mu = Mr[:, q:], likewise for V; R1 = chol; T1 = M R1^-1
  for (int side = 0; side < 2; ++side) {
    const double* G = side == 0 ? Gr : Gc;
    const double* M = side == 0 ? Mr : Mc;
    const int off = side == 0 ? q : p;
    double* R1 = sm + (side == 0 ? sR1u : sR1v) * SLOT;
    double* T1 = sm + (side == 0 ? sT1u : sT1v) * SLOT;
    // W0 = G M[:, off:off+d]  (k x d)
    for (int idx = lane; idx < k * d; idx += 64) {
      const int a = idx / d, c = idx % d;
      double s = 0.0;
      for (int t = 0; t < k; ++t) s += G[a * KM + t] * M[t * KM + off + c];
      W0[a * KM + c] = s;
    }
    __syncthreads();
    for (int idx = lane; idx < SLOT; idx += 64) W1[idx] = 0.0;
    __syncthreads();
    for (int idx = lane; idx < d * d; idx += 64) {
      const int a = idx / d, c = idx % d;
      double s = 0.0;
      for (int t = 0; t < k; ++t) s += M[t * KM + off + a] * W0[t * KM + c];
      W1[a * KM + c] = s;
    }
    __syncthreads();
    ok = chol_upper(W1, R1, d) && ok;
    for (int idx = lane; idx < SLOT; idx += 64) T1[idx] = 0.0;
    __syncthreads();
    for (int idx = lane; idx < k * d; idx += 64) {
      const int a = idx / d, c = idx % d;
      T1[a * KM + c] = M[a * KM + off + c];
    }
    __syncthreads();
    right_solve_upper(T1, k, R1, d);
  }
  if (lane == 0) status[0] = ok ? 0.0 : 1.0;
}

// Step 2: second Cholesky, core SVD, final maps F_u = Mu R_u^-1 P S, F_v = Mv R_v^-1 Q.
__global__ __launch_bounds__(64) void solve2_kernel(double* sm, int p, int q, int d,
                                                    int* err_flag) {
  const int k = p + q + d;
  const int lane = threadIdx.x;
  double* status = sm + sStatus * SLOT;
  double* W0 = sm + sW0 * SLOT;
  double* W1 = sm + sW1 * SLOT;
  double* W2 = sm + sW2 * SLOT;
  bool ok = status[0] == 0.0;
  // R = R2 R1 for both sides (stored in sR1*)
  for (int side = 0; side < 2; ++side) {
    const double* G2 = sm + (side == 0 ? sG2u : sG2v) * SLOT;
    double* R1 = sm + (side == 0 ? sR1u : sR1v) * SLOT;
    ok = chol_upper(G2, W0, d) && ok;
    matmul(W0, R1, W1, d, d, d);
    for (int idx = lane; idx < SLOT; idx += 64) R1[idx] = W1[idx];
    __syncthreads();
  }
  const double* Ru = sm + sR1u * SLOT;
  const double* Rv = sm + sR1v * SLOT;
  // C = Ru Rv'
  for (int idx = lane; idx < SLOT; idx += 64) W0[idx] = 0.0;
  __syncthreads();
  for (int idx = lane; idx < d * d; idx += 64) {
    const int i = idx / d, j = idx % d;
    double s = 0.0;
    for (int t = 0; t < d; ++t) s += Ru[i * KM + t] * Rv[j * KM + t];
    W0[i * KM + j] = s;
  }
  __syncthreads();
  double* sig = W2 + 32 * KM;   // d values in an unused part of W2
  jacobi_svd(W0, W1, sig, d);   // W0 = P S (column scaled), W1 = Q
  // order columns by decreasing singular value (selection, stable)
  __shared__ int order[64];
  if (lane == 0) {
    bool used[64];
    for (int c = 0; c < d; ++c) used[c] = false;
    for (int o = 0; o < d; ++o) {
      int best = -1;
      for (int c = 0; c < d; ++c)
        if (!used[c] && (best < 0 || sig[c] > sig[best])) best = c;
      used[best] = true;
      order[o] = best;
    }
  }
  __syncthreads();
  // F_u = Mu Ru^-1 (P S): Mu Ru^-1 = (Mu R1^-1) R2^-1 ... recompute from Mr directly
  const int offs[2] = {q, p};
  for (int side = 0; side < 2; ++side) {
    const double* M = sm + (side == 0 ? sMr : sMc) * SLOT;
    const double* Rm = side == 0 ? Ru : Rv;
    double* F = sm + (side == 0 ? sFu : sFv) * SLOT;
    for (int idx = lane; idx < SLOT; idx += 64) W2[idx] = 0.0;
    __syncthreads();
    for (int idx = lane; idx < k * d; idx += 64) {
      const int a = idx / d, c = idx % d;
      W2[a * KM + c] = M[a * KM + offs[side] + c];
    }
    __syncthreads();
    right_solve_upper(W2, k, Rm, d);
    const double* Rt = side == 0 ? W0 : W1;   // P S or Q
    for (int idx = lane; idx < k * d; idx += 64) {
      const int a = idx / d, c = idx % d;
      const int src = order[c];
      double s = 0.0;
      for (int t = 0; t < d; ++t) s += W2[a * KM + t] * Rt[t * KM + src];
      F[a * KM + c] = s;
    }
    __syncthreads();
  }
  if (lane == 0 && !ok) atomicOr(err_flag, 4);
}

// First non-zero entry of each V column in original order: key = (orig << 1) | sign.
__global__ void firstnz_kernel(const float* Pcol, int KP, int64_t m, int k, const double* Fv,
                               int d, const int* col_perm, unsigned long long* key) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * d) return;
  const int64_t j = idx / d;
  const int c = (int)(idx % d);
  double v = 0.0;
  for (int a = 0; a < k; ++a) v += (double)Pcol[j * KP + a] * Fv[a * KM + c];
  if (v != 0.0) {
    const unsigned long long kk =
        ((unsigned long long)col_perm[j] << 1) | (v < 0.0 ? 1ull : 0ull);
    atomicMin(key + c, kk);
  }
}

__global__ void init_keys_kernel(unsigned long long* key, int d) {
  if ((int)threadIdx.x < d) key[threadIdx.x] = ~0ull;
}

__global__ void sign_kernel(double* sm, const unsigned long long* key, int k, int d) {
  double* Fu = sm + sFu * SLOT;
  double* Fv = sm + sFv * SLOT;
  const int c = threadIdx.x;
  if (c >= d) return;
  if (key[c] != ~0ull && (key[c] & 1ull)) {
    for (int a = 0; a < k; ++a) {
      Fu[a * KM + c] = -Fu[a * KM + c];
      Fv[a * KM + c] = -Fv[a * KM + c];
    }
  }
}

// out_first[orig][c] = P_i . Mfirst[:, c0 + c] (nf columns), out_lat[orig][c] = P_i . F[:, c]
__global__ void apply_kernel(const float* P, int KP, int64_t rows, int k, const double* Mm,
                             int c0, int nf, const double* F, int d, const int* perm,
                             float* out_first, float* out_lat) {
  const int w = nf + d;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * w) return;
  const int64_t i = idx / w;
  const int c = (int)(idx % w);
  const float* pr = P + i * KP;
  double s = 0.0;
  if (c < nf) {
    for (int a = 0; a < k; ++a) s += (double)pr[a] * Mm[a * KM + c0 + c];
    if (out_first) out_first[(int64_t)perm[i] * nf + c] = (float)s;
  } else {
    const int cc = c - nf;
    for (int a = 0; a < k; ++a) s += (double)pr[a] * F[a * KM + cc];
    if (out_lat) out_lat[(int64_t)perm[i] * d + cc] = (float)s;
  }
}

}  // namespace

size_t postprocess_scratch_doubles(int64_t n, int64_t m, int KP, int nblocks) {
  (void)KP; (void)nblocks;
  const size_t need = (size_t)(kGramBlocks + kSlots) * SLOT + 64;
  const size_t setp = (size_t)((n + m) * 64 / 2 + 16);
  return need > setp ? need : setp;
}

hipError_t launch_postprocess(const PostArgs& a, hipStream_t s) {
  const int k = a.p + a.q + a.d;
  double* part = a.gram_part;
  double* sm = a.gram_part + (size_t)kGramBlocks * SLOT;
  unsigned long long* keys = reinterpret_cast<unsigned long long*>(sm + kSlots * SLOT);
  const int sum_grid = (SLOT + 255) / 256;
  hipLaunchKernelGGL(gram_kernel, dim3(kGramBlocks), dim3(256), 0, s, a.Prow, a.KP, a.n, k,
                     (const double*)nullptr, 0, part);
  hipLaunchKernelGGL(sum_slots_kernel, dim3(sum_grid), dim3(256), 0, s, part, kGramBlocks,
                     sm + sGr * SLOT);
  hipLaunchKernelGGL(gram_kernel, dim3(kGramBlocks), dim3(256), 0, s, a.Pcol, a.KP, a.m, k,
                     (const double*)nullptr, 0, part);
  hipLaunchKernelGGL(sum_slots_kernel, dim3(sum_grid), dim3(256), 0, s, part, kGramBlocks,
                     sm + sGc * SLOT);
  hipLaunchKernelGGL(solve1_kernel, dim3(1), dim3(64), 0, s, sm, a.p, a.q, a.d);
  hipLaunchKernelGGL(gram_kernel, dim3(kGramBlocks), dim3(256), 0, s, a.Prow, a.KP, a.n, k,
                     (const double*)(sm + sT1u * SLOT), a.d, part);
  hipLaunchKernelGGL(sum_slots_kernel, dim3(sum_grid), dim3(256), 0, s, part, kGramBlocks,
                     sm + sG2u * SLOT);
  hipLaunchKernelGGL(gram_kernel, dim3(kGramBlocks), dim3(256), 0, s, a.Pcol, a.KP, a.m, k,
                     (const double*)(sm + sT1v * SLOT), a.d, part);
  hipLaunchKernelGGL(sum_slots_kernel, dim3(sum_grid), dim3(256), 0, s, part, kGramBlocks,
                     sm + sG2v * SLOT);
  hipLaunchKernelGGL(solve2_kernel, dim3(1), dim3(64), 0, s, sm, a.p, a.q, a.d, a.err_flag);
  hipLaunchKernelGGL(init_keys_kernel, dim3(1), dim3(64), 0, s, keys, a.d);
  const int64_t md = a.m * a.d;
  hipLaunchKernelGGL(firstnz_kernel, dim3((unsigned)((md + 255) / 256)), dim3(256), 0, s,
                     a.Pcol, a.KP, a.m, k, (const double*)(sm + sFv * SLOT), a.d, a.col_perm,
                     keys);
  hipLaunchKernelGGL(sign_kernel, dim3(1), dim3(64), 0, s, sm, keys, k, a.d);
  const int64_t nw = a.n * (a.q + a.d), mw = a.m * (a.p + a.d);
  hipLaunchKernelGGL(apply_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, a.Prow,
                     a.KP, a.n, k, (const double*)(sm + sMr * SLOT), 0, a.q,
                     (const double*)(sm + sFu * SLOT), a.d, a.row_perm, a.A, a.U);
  hipLaunchKernelGGL(apply_kernel, dim3((unsigned)((mw + 255) / 256)), dim3(256), 0, s, a.Pcol,
                     a.KP, a.m, k, (const double*)(sm + sMc * SLOT), 0, a.p,
                     (const double*)(sm + sFv * SLOT), a.d, a.col_perm, a.B, a.V);
  return hipGetLastError();
}

}  // namespace gmf
