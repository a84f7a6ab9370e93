// Device kernels (gfx950, wave64) of the Riesz-map PCG solver.
//
// Hot path per PCG iteration (Sec. 7.1, with the preconditioners of Sec. 6):
//  * apply_A: y = sum_T P_T^T (sum_q w_{T,q} R_q) P_T x in three stages: a
//    gather of the cell vectors x_T into MFMA fragment order, the contraction
//    over the stacked reference matrices as a GEMM with M = n_loc,
//    K = Q n_loc, N = cells on FP64 (or FP32) MFMA 16x16x4, the weight
//    w_{T,q} multiplying the B fragment in registers, and an assembly that
//    sums, per dof, its (cell, row) entries in a fixed order (no atomics).
//  * apply_P: point-Jacobi on the interior block; per interface patch the
//    packed (segmented) symmetric inverse streamed from HBM against the
//    gathered residual, the mirrored products kept in registers; the Whitney
//    coarse solve as a tiled packed symmetric matrix-vector product, or the
//    multigrid V-cycle on W^k.
//  * Krylov vectors: fused axpy updates with block reductions, scalars kept
//    on the device and a done flag that makes every later kernel a no-op.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "kernels.hpp"

namespace rz {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// one 64-bit DPP lane move (gfx9 DPP controls: quad_perm, row_mirror ...)
template <int CTRL>
__device__ inline double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// sum over aligned groups of L lanes (L = 16, 32, 64); every lane of a group
// gets the group sum.  Within a 16-lane row: quad_perm [1,0,3,2], quad_perm
// [2,3,0,1], row_half_mirror, row_mirror; across rows: lane permutes.  Must
// be called with all 64 lanes active.
template <int CTRL>
__device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int L, typename C>
__device__ inline C group_sum(C v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  v += dpp_mov<0x140>(v);
  if (L >= 32) v += __shfl_xor(v, 16, 64);
  if (L >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// stored inverse entries -> the patch kernels' arithmetic type (uint16_t
// holds bfloat16 bits, which widen exactly to FP32)
__device__ inline double widen(double v) { return v; }
__device__ inline double widen(float v) { return double(v); }
__device__ inline float widen(uint16_t v) { return __uint_as_float(uint32_t(v) << 16); }
__device__ inline double to_f64(double v) { return v; }
__device__ inline double to_f64(float v) { return double(v); }
template <typename T>
__device__ inline T from_f64(double v);
template <>
__device__ inline float from_f64<float>(double v) { return float(v); }
template <>
__device__ inline uint16_t from_f64<uint16_t>(double v) {
  // round to nearest even on the float32 bits (finite values)
  const uint32_t b = __float_as_uint(float(v));
  return uint16_t((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

// deterministic block sum of 256 threads; result valid in every thread
__device__ inline double block_sum256(double v, double *sm4) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sm4[wave] = v;
  __syncthreads();
  return (sm4[0] + sm4[1]) + (sm4[2] + sm4[3]);
}

inline unsigned grid_for(int64_t n, int bs, unsigned cap = 1u << 20) {
  int64_t g = (n + bs - 1) / bs;
  if (g < 1) g = 1;
  return unsigned(g > cap ? cap : g);
}

// ------------------------------------------------------------------ setup
// w_{T,q} of the stacked form for one cell per thread.  k selects the pullback
// (eq:pullback-3d-def): 0 identity (H(grad)), 1 covariant Piola (H(curl)),
// 2 contravariant Piola (H(div), also the 2D RT_p whose form degree is 1).
__global__ void k_weights(int d, int k, int64_t nc, const double *__restrict__ X, const double *__restrict__ Einv,
                          double alpha, double beta, double *__restrict__ w, int Q) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const double *x = X + c * (d + 1) * d;
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int a = 0; a < d; ++a)
    for (int m = 0; m < d; ++m) {
      double s = 0;
      for (int b = 0; b < d; ++b) s += (x[(b + 1) * d + a] - x[a]) * Einv[b * d + m];
      J[a][m] = s;
    }
  double det, Ji[3][3];
  if (d == 3) {
    det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    const double id = 1.0 / det;
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  } else {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double id = 1.0 / det;
    Ji[0][0] = J[1][1] * id;
    Ji[0][1] = -J[0][1] * id;
    Ji[1][0] = -J[1][0] * id;
    Ji[1][1] = J[0][0] * id;
  }
  const double s = fabs(det);
  double G[3][3], H[3][3];  // G = J^{-1} J^{-T}, H = J^T J
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double g = 0, h = 0;
      for (int m = 0; m < d; ++m) {
        g += Ji[a][m] * Ji[b][m];
        h += J[m][a] * J[m][b];
      }
      G[a][b] = g;
      H[a][b] = h;
    }
  const int pa3[6] = {0, 1, 2, 0, 0, 1}, pb3[6] = {0, 1, 2, 1, 2, 2};
  const int pa2[3] = {0, 1, 0}, pb2[3] = {0, 1, 1};
  const int np = d == 3 ? 6 : 3;
  const int *pa = d == 3 ? pa3 : pa2, *pb = d == 3 ? pb3 : pb2;
  double *wc = w + c * Q;
  if (k == 0) {
    wc[0] = beta * s;
    for (int i = 0; i < np; ++i) wc[1 + i] = alpha * s * G[pa[i]][pb[i]];
  } else if (k == 1) {
    for (int i = 0; i < np; ++i) wc[i] = beta * s * G[pa[i]][pb[i]];
    if (d == 3)
      for (int i = 0; i < np; ++i) wc[np + i] = alpha * H[pa[i]][pb[i]] / s;  // J curl / det J
    else
      wc[np] = alpha / s;  // the 2D rot is a scalar: rot / det J
  } else {
    for (int i = 0; i < np; ++i) wc[i] = beta * H[pa[i]][pb[i]] / s;
    wc[np] = alpha / s;
  }
}

__global__ void k_interior_diag(int64_t nc, int n, int Q, const double *__restrict__ R, const double *__restrict__ w,
                                const int32_t *__restrict__ cd, const int32_t *__restrict__ loc, int nloc,
                                int64_t offI, double *__restrict__ dinv) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nc * nloc) return;
  const int64_t c = t / nloc;
  const int li = loc[t - c * nloc];
  double s = 0;
  for (int q = 0; q < Q; ++q) s += w[c * Q + q] * R[(size_t(q) * n + li) * n + li];
  dinv[cd[c * n + li] - offI] = 1.0 / s;
}

__global__ void k_pad_identity(int64_t B, int N, const int32_t *__restrict__ sizes, double *__restrict__ A) {
  const int64_t b = blockIdx.x;
  for (int i = sizes[b] + threadIdx.x; i < N; i += blockDim.x) A[(b * N + i) * N + i] = 1.0;
}

__global__ void k_patch_assemble(const int32_t *__restrict__ item_patch, const int32_t *__restrict__ item_cell,
                                 const int64_t *__restrict__ item_trip, const int32_t *__restrict__ tr_col,
                                 const int32_t *__restrict__ tr_loc, const double *__restrict__ tr_coef, int n, int Q,
                                 const double *__restrict__ R, const double *__restrict__ w, int N,
                                 double *__restrict__ A) {
  const int64_t it = blockIdx.x;
  const int64_t t0 = item_trip[it], cnt = item_trip[it + 1] - t0;
  const int64_t c = item_cell[it];
  double *Ap = A + int64_t(item_patch[it]) * N * N;
  double wq[16];
  for (int q = 0; q < Q; ++q) wq[q] = w[c * Q + q];
  for (int64_t pi = threadIdx.x; pi < cnt * cnt; pi += blockDim.x) {
    const int64_t a = t0 + pi / cnt, b = t0 + pi % cnt;
    const int la = tr_loc[a], lb = tr_loc[b];
    double s = 0;
    for (int q = 0; q < Q; ++q) s += wq[q] * R[(size_t(q) * n + la) * n + lb];
    atomicAdd(&Ap[int64_t(tr_col[a]) * N + tr_col[b]], tr_coef[a] * tr_coef[b] * s);
  }
}

// ---- batched blocked Cholesky (lower) and inverse, block size 32
constexpr int BS = 32;

// acc += op(A) op(B) for the 16 x 16 quadrant (wave >> 1, wave & 1) of a
// 32 x 32 tile product over K = 32 (FP64 MFMA 16x16x4; A and B are LDS
// tiles, op = transpose where asked).  acc element v of lane l is row
// 16 (wave >> 1) + l/16 + 4v, column 16 (wave & 1) + l%16.
template <bool TA, bool TB>
__device__ inline void tile_mfma(const double (*A)[BS + 1], const double (*B)[BS + 1], d4 &acc) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ri = 16 * (wave >> 1) + (lane & 15), cj = 16 * (wave & 1) + (lane & 15), lk = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < BS; k0 += 4) {
    const double a = TA ? A[k0 + lk][ri] : A[ri][k0 + lk];
    const double b = TB ? B[cj][k0 + lk] : B[k0 + lk][cj];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
}

__global__ void k_chol_diag(int N, int kb, double *__restrict__ A, int *__restrict__ status) {
  __shared__ double L[BS][BS + 1];
  __shared__ double piv;
  double *M = A + int64_t(blockIdx.x) * N * N;
  const int o = kb * BS;
  for (int t = threadIdx.x; t < BS * BS; t += blockDim.x) {
    const int i = t / BS, j = t % BS;
    L[i][j] = M[int64_t(o + i) * N + o + j];
  }
  __syncthreads();
  for (int j = 0; j < BS; ++j) {
    if (threadIdx.x == 0) {
      double a = L[j][j];
      if (!(a > 0.0)) {
        atomicExch(status, 1);
        a = 1.0;
      }
      piv = sqrt(a);
      L[j][j] = piv;
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < BS; i += blockDim.x) L[i][j] /= piv;
    __syncthreads();
    for (int t = threadIdx.x; t < BS * BS; t += blockDim.x) {
      const int i = t / BS, m = t % BS;
      if (i > j && m > j && m <= i) L[i][m] -= L[i][j] * L[m][j];
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < BS * BS; t += blockDim.x) {
    const int i = t / BS, j = t % BS;
    M[int64_t(o + i) * N + o + j] = j <= i ? L[i][j] : 0.0;
  }
}

__global__ void k_chol_panel(int N, int kb, double *__restrict__ A) {
  __shared__ double L[BS][BS + 1];
  __shared__ double X[BS][BS + 1];
  double *M = A + int64_t(blockIdx.y) * N * N;
  const int o = kb * BS, ob = (kb + 1 + blockIdx.x) * BS;
  for (int t = threadIdx.x; t < BS * BS; t += blockDim.x) {
    const int i = t / BS, j = t % BS;
    L[i][j] = M[int64_t(o + i) * N + o + j];
    X[i][j] = M[int64_t(ob + i) * N + o + j];
  }
  __syncthreads();
  // X L^T = A_block, row by row
  if (threadIdx.x < BS) {
    const int r = threadIdx.x;
    for (int c = 0; c < BS; ++c) {
      double s = X[r][c];
      for (int m = 0; m < c; ++m) s -= X[r][m] * L[c][m];
      X[r][c] = s / L[c][c];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < BS * BS; t += blockDim.x) {
    const int i = t / BS, j = t % BS;
    M[int64_t(ob + i) * N + o + j] = X[i][j];
  }
}

__device__ inline void tri_decode(int64_t t, int &i, int &j) {
  int ii = int((sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
  while (int64_t(ii + 1) * (ii + 2) / 2 <= t) ++ii;
  while (int64_t(ii) * (ii + 1) / 2 > t) --ii;
  i = ii;
  j = int(t - int64_t(ii) * (ii + 1) / 2);
}

__global__ void k_chol_update(int N, int kb, double *__restrict__ A) {
  __shared__ double La[BS][BS + 1];
  __shared__ double Lb[BS][BS + 1];
  double *M = A + int64_t(blockIdx.y) * N * N;
  int i_, j_;
  tri_decode(blockIdx.x, i_, j_);
  const int o = kb * BS, oi = (kb + 1 + i_) * BS, oj = (kb + 1 + j_) * BS;
  for (int t = threadIdx.x; t < BS * BS; t += blockDim.x) {
    const int i = t / BS, j = t % BS;
    La[i][j] = M[int64_t(oi + i) * N + o + j];
    Lb[i][j] = M[int64_t(oj + i) * N + o + j];
  }
  __syncthreads();
  d4 acc = {0, 0, 0, 0};
  tile_mfma<false, true>(La, Lb, acc);  // La Lb^T
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 16 * (wave >> 1) + (lane >> 4) + 4 * v, j = 16 * (wave & 1) + (lane & 15);
    M[int64_t(oi + i) * N + oj + j] -= acc[v];
  }
}

// X = L^{-1}, lower triangular, by diagonal offsets s = ib - jb.  s = 0: the
// diagonal tiles X[ib][ib] = L[ib][ib]^{-1} by forward substitution (one
// column per thread).  s >= 1: X[ib][jb] = -X[ib][ib] sum_{jb <= mb < ib}
// L[ib][mb] X[mb][jb], the sum and the product on MFMA; when a step has few
// tiles (a large single matrix) the sum is split over blocks and the partial
// tiles are added in a fixed order by the finishing kernel.
__global__ void k_trtri_diag(int N, const double *__restrict__ A, double *__restrict__ X) {
  __shared__ double Lt[BS][BS + 1];
  __shared__ double S[BS][BS + 1];
  const int ib = blockIdx.x;
  const double *M = A + int64_t(blockIdx.y) * N * N;
  double *Y = X + int64_t(blockIdx.y) * N * N;
  const int oi = ib * BS;
  for (int t = threadIdx.x; t < BS * BS; t += blockDim.x) {
    const int i = t / BS, j = t % BS;
    Lt[i][j] = M[int64_t(oi + i) * N + oi + j];
    S[i][j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  if (threadIdx.x < BS) {
    const int c = threadIdx.x;
    for (int r = 0; r < BS; ++r) {
      double v = S[r][c];
      for (int m = 0; m < r; ++m) v -= Lt[r][m] * S[m][c];
      S[r][c] = v / Lt[r][r];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < BS * BS; t += blockDim.x) {
    const int i = t / BS, j = t % BS;
    Y[int64_t(oi + i) * N + oi + j] = S[i][j];
  }
}

// acc += sum_{m0 <= mb < m1} L[ib][mb] X[mb][jb] (this wave's quadrant)
__device__ inline void trtri_sum(int N, const double *M, const double *Y, int ib, int jb, int m0, int m1,
                                 double (*Lt)[BS + 1], double (*Xt)[BS + 1], d4 &acc) {
  const int oi = ib * BS, oj = jb * BS;
  for (int mb = m0; mb < m1; ++mb) {
    __syncthreads();
    for (int t = threadIdx.x; t < BS * BS; t += blockDim.x) {
      const int i = t / BS, j = t % BS;
      Lt[i][j] = M[int64_t(oi + i) * N + mb * BS + j];
      Xt[i][j] = Y[int64_t(mb * BS + i) * N + oj + j];
    }
    __syncthreads();
    tile_mfma<false, false>(Lt, Xt, acc);
  }
}

// X[ib][jb] = X[ib][ib] (-acc) on MFMA (Dt, St: LDS tiles, free on entry)
__device__ inline void trtri_finish(int N, double *Y, int ib, int jb, const d4 &acc, double (*Dt)[BS + 1],
                                    double (*St)[BS + 1]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int oi = ib * BS, oj = jb * BS;
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 16 * (wave >> 1) + (lane >> 4) + 4 * v, j = 16 * (wave & 1) + (lane & 15);
    St[i][j] = -acc[v];
  }
  for (int t = threadIdx.x; t < BS * BS; t += blockDim.x) {
    const int i = t / BS, j = t % BS;
    Dt[i][j] = Y[int64_t(oi + i) * N + oi + j];
  }
  __syncthreads();
  d4 out = {0, 0, 0, 0};
  tile_mfma<false, false>(Dt, St, out);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 16 * (wave >> 1) + (lane >> 4) + 4 * v, j = 16 * (wave & 1) + (lane & 15);
    Y[int64_t(oi + i) * N + oj + j] = out[v];
  }
}

// step s >= 1, whole sums: grid (NB - s, B)
__global__ void k_trtri_step(int N, int s, const double *__restrict__ A, double *__restrict__ X) {
  __shared__ double Lt[BS][BS + 1];
  __shared__ double Xt[BS][BS + 1];
  const int NB = N / BS;
  const int jb = blockIdx.x, ib = jb + s;
  if (ib >= NB) return;
  const double *M = A + int64_t(blockIdx.y) * N * N;
  double *Y = X + int64_t(blockIdx.y) * N * N;
  d4 acc = {0, 0, 0, 0};
  trtri_sum(N, M, Y, ib, jb, jb, ib, Lt, Xt, acc);
  trtri_finish(N, Y, ib, jb, acc, Lt, Xt);
}

// step s >= 1, split sums: grid (NB - s, nK, B); partial kc covers mb in
// [jb + kc KC, min(ib, jb + (kc + 1) KC)), stored in accumulator order
__global__ void k_trtri_part(int N, int s, int KC, int nK, const double *__restrict__ A,
                             const double *__restrict__ X, double *__restrict__ P) {
  __shared__ double Lt[BS][BS + 1];
  __shared__ double Xt[BS][BS + 1];
  const int NB = N / BS;
  const int jb = blockIdx.x, ib = jb + s, kc = blockIdx.y;
  if (ib >= NB) return;
  const double *M = A + int64_t(blockIdx.z) * N * N;
  const double *Y = X + int64_t(blockIdx.z) * N * N;
  const int m0 = jb + kc * KC, m1 = min(ib, m0 + KC);
  d4 acc = {0, 0, 0, 0};
  trtri_sum(N, M, Y, ib, jb, m0, m1, Lt, Xt, acc);
  double *out = P + ((int64_t(blockIdx.z) * (NB - s) + jb) * nK + kc) * (BS * BS) + threadIdx.x * 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) out[v] = acc[v];
}

// step s >= 1 after k_trtri_part: the partials added in kc order, then the
// product with the diagonal inverse; grid (NB - s, B)
__global__ void k_trtri_fin(int N, int s, int nK, const double *__restrict__ P, double *__restrict__ X) {
  __shared__ double Dt[BS][BS + 1];
  __shared__ double St[BS][BS + 1];
  const int NB = N / BS;
  const int jb = blockIdx.x, ib = jb + s;
  if (ib >= NB) return;
  double *Y = X + int64_t(blockIdx.y) * N * N;
  const double *in = P + (int64_t(blockIdx.y) * (NB - s) + jb) * nK * (BS * BS) + threadIdx.x * 4;
  d4 acc = {0, 0, 0, 0};
  for (int kc = 0; kc < nK; ++kc)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] += in[int64_t(kc) * (BS * BS) + v];
  trtri_finish(N, Y, ib, jb, acc, Dt, St);
}

// A^{-1} = X^T X with X = L^{-1} lower triangular: tile (I >= J)
__global__ void k_lauum(int N, const double *__restrict__ X, double *__restrict__ A) {
  __shared__ double Xa[BS][BS + 1];
  __shared__ double Xb[BS][BS + 1];
  const int NB = N / BS;
  int I, J;
  tri_decode(blockIdx.x, I, J);
  const double *Y = X + int64_t(blockIdx.y) * N * N;
  double *M = A + int64_t(blockIdx.y) * N * N;
  d4 acc = {0, 0, 0, 0};
  for (int K = I; K < NB; ++K) {
    __syncthreads();
    for (int t = threadIdx.x; t < BS * BS; t += blockDim.x) {
      const int i = t / BS, j = t % BS;
      Xa[i][j] = Y[int64_t(K * BS + i) * N + I * BS + j];
      Xb[i][j] = Y[int64_t(K * BS + i) * N + J * BS + j];
    }
    __syncthreads();
    tile_mfma<true, false>(Xa, Xb, acc);  // X[K][I]^T X[K][J]
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 16 * (wave >> 1) + (lane >> 4) + 4 * v, j = 16 * (wave & 1) + (lane & 15);
    M[int64_t(I * BS + i) * N + J * BS + j] = acc[v];
    M[int64_t(J * BS + j) * N + I * BS + i] = acc[v];
  }
}

// Segmented upper layout of a symmetric m x m patch inverse (E elements per
// segment, mS = m rounded up to E): row i holds the columns [s_i, mS) with
// s_i = E floor(i / E); entries left of the diagonal and right of m are zero
// and the diagonal is stored halved, so that the row products (j >= i) and the
// mirrored column products (j >= i) together apply the full matrix.  Every
// row is a whole number of E-element segments, aligned to E elements.
__device__ __host__ inline int64_t seg_row_off(int64_t i, int64_t mS, int E) {
  const int64_t b = i / E;
  return E * (b * mS - E * b * (b - 1) / 2) + (i - b * E) * (mS - b * E);
}

__global__ void k_pack_seg(int N, int E, const int32_t *__restrict__ sizes, const int64_t *__restrict__ off,
                           const double *__restrict__ A, double *__restrict__ P) {
  const int64_t b = blockIdx.x;
  const int m = sizes[b];
  const int mS = (m + E - 1) / E * E;
  const double *M = A + b * N * N;
  double *out = P + off[b];
  for (int i = 0; i < m; ++i) {
    const int64_t ro = seg_row_off(i, mS, E);
    const int si = i / E * E;
    for (int k = si + threadIdx.x; k < mS; k += blockDim.x) {
      double v = 0.0;
      if (k >= i && k < m) v = (k == i ? 0.5 : 1.0) * M[int64_t(i) * N + k];
      out[ro + k - si] = v;
    }
  }
}

// Element (r, c) of a 64 x 64 coarse tile: wave ty = r / 16 of the reading
// block loads rows 16 ty .. 16 ty + 15 as eight coalesced pairs (rows 2q,
// 2q + 1 of its slice) per lane c.
__device__ __host__ inline int ctile_idx(int r, int c) { return (r >> 4) * 1024 + ((r & 15) >> 1) * 128 + c * 2 + (r & 1); }

// the folded layout (see kFoldMin) of the upper triangles of the inverses
__global__ void k_pack_fold(int N, const int32_t *__restrict__ sizes, const int64_t *__restrict__ off,
                            const double *__restrict__ A, double *__restrict__ P) {
  const int64_t b = blockIdx.x;
  const int m = sizes[b];
  const int h = (m + 1) / 2, hP = fold_hp(m, 8);
  const double *M = A + b * N * N;
  double *out = P + off[b];
  const int64_t total = int64_t(h + 1) * 2 * hP;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int k = int(e / (2 * hP)), q = int(e % (2 * hP));
    double v = 0.0;
    if (q < hP) {
      const int p = q;
      if (p >= k) {
        if (p < h) v = (p == k ? 0.5 : 1.0) * M[int64_t(k) * N + p];
      } else if (h + k - 1 < m) {
        v = (p == k - 1 ? 0.5 : 1.0) * M[int64_t(h + p) * N + h + k - 1];
      }
    } else {
      const int p = q - hP;
      if (k < h && h + p < m) v = M[int64_t(k) * N + h + p];
    }
    out[e] = v;
  }
}

__global__ void k_pack_tiles(int N, int n, int NT, const double *__restrict__ A, double *__restrict__ T) {
  const int64_t t = blockIdx.x;
  // decode upper tile (I <= J): t = I*NT - I(I-1)/2 + (J - I)
  int I = 0;
  while (int64_t(I + 1) * NT - int64_t(I + 1) * I / 2 <= t) ++I;
  const int J = int(t - (int64_t(I) * NT - int64_t(I) * (I - 1) / 2)) + I;
  double *out = T + t * 64 * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    const int r = e / 64, c = e % 64;
    const int gi = I * 64 + r, gj = J * 64 + c;
    out[ctile_idx(r, c)] = (gi < n && gj < n) ? A[int64_t(gi) * N + gj] : 0.0;
  }
}

// -------------------------------------------------------------- apply_A
// ---- Operator apply in three stages: cell gather, GEMM, assembly (FP64, or
// FP32 with FP32 tables: T is the type of the cell vectors and the MFMA).
// Cell-local vectors in MFMA fragment order (ncp = cells rounded up to 256; per
// column KP ncp entries of Xc and NP ncp of Yc):
//   Xc[(kb ncp + c16) 4 + kk 16 + ci] = x[cell_dofs[cell][4 kb + kk]]
//     (cell = c16 + ci, c16 a multiple of 16; zero beyond n and for padding
//     cells): lane l of a B fragment reads kk = l / 16, ci = l % 16 (the
//     same for the FP64 and FP32 16x16x4 MFMA);
//   Yc[yc_index(ncp, cell, r)] = (A_T x_T)_r: row rr = r % 16 of row block
//     mb = r / 16 and cell c16 + ci at (mb ncp + c16) 16 + 64 (rr / 4) +
//     16 (rr % 4) + ci, 16 rows x 16 cells per (mb, c16) block.  The FP64
//     accumulator element v of lane l (row l/16 + 4v, cell l % 16) lands at
//     64 v + l; the FP32 one (row 4 (l/16) + v) at 64 (l/16) + 16 v + l % 16.
template <typename T>
__global__ void k_gather_cells(int n, int KP, int64_t nc, int64_t ncp, int kb0, int kb1,
                               const int32_t *__restrict__ cd, const double *__restrict__ x, int64_t ldx,
                               T *__restrict__ Xc, const PcgState *st, const uint8_t *__restrict__ dm) {
  const int c = blockIdx.y;
  if (st && st[c].done) return;
  const double *xc = x + int64_t(c) * ldx;
  T *X = Xc + int64_t(c) * KP * ncp + int64_t(kb0) * ncp * 4;
  const int64_t nblk = ncp / 16;
  const int64_t total = int64_t(kb1 - kb0) * ncp * 4;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int ci = int(t & 15), kk = int((t >> 4) & 3);
    const int64_t b = t >> 6;
    const int64_t cell = (b % nblk) * 16 + ci;
    const int k = (kb0 + int(b / nblk)) * 4 + kk;
    T v = T(0);
    if (cell < nc && k < n) {
      const int32_t g = cd[cell * n + k];
      if (!dm || !dm[g]) v = T(xc[g]);
    }
    X[t] = v;
  }
}

__device__ inline d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
typedef float f4 __attribute__((ext_vector_type(4)));
__device__ inline f4 mfma16x16x4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Yc = sum_q w_q R_q Xc over the k-blocks [kb0, kb1), per cell: one wave owns
// a 16-row block of 16 NB cells; per k-step the A fragments of all Q
// reference matrices and the B fragments (w_q x) are in registers, and the
// next k-step's are loaded before the current MFMAs.  All loads are plain
// (no indirection), so the prefetch is never serialised behind a dependent
// load.
template <typename T, int Q, int NB, bool FULL>
__global__ __launch_bounds__(256) void k_apply_A(int mb0, int KB, int kb0_, int kb1_, int64_t nc, int64_t ncp,
                                                 const T *__restrict__ Af, const T *__restrict__ w,
                                                 const T *__restrict__ Xc, T *__restrict__ Yc, int KP,
                                                 int NP, const PcgState *st) {
  typedef T acc_t __attribute__((ext_vector_type(4)));
  if (st && st[blockIdx.z].done) return;
  // the k-block range: all of them, or the columns of a restricted apply
  const int kb0 = FULL ? 0 : kb0_, kb1 = FULL ? KB : kb1_;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // the four waves of a block share the row block (and so the A fragments,
  // which the vector L1 then serves once) and take consecutive cell groups
  const int mb = mb0 + blockIdx.y;  // row blocks from mb0 (a row-restricted apply starts later)
  const int li = lane & 15, lk = lane >> 4;
  const T *X = Xc + int64_t(blockIdx.z) * KP * ncp + lane;
  T *Y = Yc + int64_t(blockIdx.z) * NP * ncp;
  const int64_t cell0 = (int64_t(blockIdx.x) * 4 + wave) * (16 * NB);
  T wv[NB][Q];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int64_t c = cell0 + nb * 16 + li;
#pragma unroll
    for (int q = 0; q < Q; ++q) wv[nb][q] = c < nc ? w[c * Q + q] : T(0);
  }
  acc_t acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = acc_t{0, 0, 0, 0};
  const T *Ab = Af + size_t(mb) * KB * Q * 64 + lane;
  // fragments of k-block kb: the A fragments of all Q matrices and the B
  // fragments of cells cell0 + 16 nb .. + 15 (64 consecutive entries each)
  auto load = [&](int kb, T *a, T *xv) {
    const T *An = Ab + size_t(kb) * Q * 64;
#pragma unroll
    for (int q = 0; q < Q; ++q) a[q] = An[q * 64];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) xv[nb] = X[(int64_t(kb) * ncp + cell0 + nb * 16) * 4];
  };
  auto step = [&](const T *a, const T *xv) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma16x16x4(a[q], wv[nb][q] * xv[nb], acc[nb]);
  };
  // two register sets in turn: the loads of one k-block are in flight while
  // the MFMAs of the other run (no register copies between steps)
  // (scheduling barriers keep each set's loads ahead of the other's MFMAs)
  T aA[Q], xA[NB], aB[Q], xB[NB];
  load(kb0, aA, xA);
  int jb = kb0;
  for (; jb + 1 < kb1; jb += 2) {
    load(jb + 1, aB, xB);
    __builtin_amdgcn_sched_barrier(0);
    step(aA, xA);
    __builtin_amdgcn_sched_barrier(0);
    load(jb + 2 < kb1 ? jb + 2 : kb1 - 1, aA, xA);  // unconditional: keeps the load waits exact
    __builtin_amdgcn_sched_barrier(0);
    step(aB, xB);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (jb < kb1) step(aA, xA);
  // accumulator layouts: FP64 16x16x4, lane l, element v holds row l/16 + 4v
  // (64 consecutive entries per (nb, v)); FP32, row 4 (l/16) + v (16-entry
  // runs); column (cell) l%16 in both
  const int off = sizeof(T) == 8 ? lane : 64 * (lane >> 4) + li;
  const int vstep = sizeof(T) == 8 ? 64 : 16;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int v = 0; v < 4; ++v) Y[(int64_t(mb) * ncp + cell0 + nb * 16) * 16 + off + vstep * v] = acc[nb][v];
}

// y[i] (+)= alpha sum over the (cell, local row) pairs of dof i of Yc, in
// FP64 and a fixed order (deterministic, no atomics), i in [d0, d1); with
// xclr, also x[i] = 0 (the gather that read x has completed)
template <typename T>
__global__ void k_assemble(int64_t d0, int64_t d1, const int64_t *__restrict__ ptr, const int32_t *__restrict__ ent,
                           int64_t ystride, const T *__restrict__ Yc, double *__restrict__ y, int64_t ldy,
                           double alpha, int overwrite, double *__restrict__ xclr, int64_t ldx, const PcgState *st,
                           const uint8_t *__restrict__ dm) {
  const int c = blockIdx.y;
  if (st && st[c].done) return;
  const T *Y = Yc + int64_t(c) * ystride;
  double *yc = y + int64_t(c) * ldy;
  double *xc = xclr ? xclr + int64_t(c) * ldx : nullptr;
  for (int64_t i = d0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < d1; i += int64_t(gridDim.x) * blockDim.x) {
    if (dm && dm[i]) {  // a removed dof: the row of the restricted operator is zero
      if (overwrite) yc[i] = 0.0;
      if (xc) xc[i] = 0.0;
      continue;
    }
    double sum = 0.0;
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) sum += double(Y[ent[e]]);
    yc[i] = overwrite ? alpha * sum : yc[i] + alpha * sum;
    if (xc) xc[i] = 0.0;
  }
}


__global__ void k_to_float(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    b[i] = float(a[i]);
}

// x += d per column (refinement update)
__global__ void k_axpy_m(int64_t n, const double *__restrict__ d, double *__restrict__ x, int64_t ldx) {
  const int c = blockIdx.y;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    x[c * ldx + i] += d[c * n + i];
}

// Streams of more than 192 MiB (three quarters of the 256 MiB last-level
// cache) are read with non-temporal loads; smaller ones may stay cached
// from one apply to the next (measured over the sweep's patch sets and
// coarse inverses).
#ifndef RZ_STREAM_MB
#define RZ_STREAM_MB 192
#endif
constexpr int64_t kStreamBytes = int64_t(RZ_STREAM_MB) << 20;

// Patch solves z += R_p^T A_p^{-1} R_p r for a chunk of rows of one patch
// (NT: the rows are read with non-temporal loads, for sets too large to stay
// in the last-level cache between applies)
// and G right-hand sides (blockIdx.y), the inverse in the segmented layout
// with V-element segments (16 bytes).  A wave works on 64 / L rows at a time,
// L lanes per row; lane t owns the columns q V L + t V + [0, V) for q < NQ,
// so each segment load is contiguous across the lanes of a row.  Row products
// are summed over the L lanes (DPP); the mirrored column products stay in
// registers until the end of the chunk.  Segments left of a row's first
// stored segment or beyond the patch are not loaded.
template <int V, int L, int NQ, int G, int D, typename T, int NW, bool NT>
__global__ __launch_bounds__(64 * NW) void k_patch_seg(const int64_t *__restrict__ chunk_patch,
                                                   const int32_t *__restrict__ chunk_rows,
                                                   const int64_t *__restrict__ patch_col,
                                                   const int64_t *__restrict__ col_ent,
                                                   const int32_t *__restrict__ ent_dof,
                                                   const double *__restrict__ ent_coef,
                                                   const int64_t *__restrict__ inv_off, const T *__restrict__ inv,
                                                   const double *__restrict__ r, int64_t ldr, double *__restrict__ z,
                                                   int64_t ldz, int ncol, double scale, const PcgState *st) {
  // arithmetic: FP64 for FP64/FP32 entries; FP32 for bfloat16 entries (their
  // rounding, 2^-9, dwarfs FP32 accumulation error)
  typedef decltype(widen(T())) C;
  constexpr int RPW = 64 / L;        // rows per wave step
  constexpr int W = NQ * L * V;      // columns covered (LDS stride)
  typedef T vecV __attribute__((ext_vector_type(V)));
  const int cbase = blockIdx.y * G;
  if (st) {
    bool any = false;
    for (int g = 0; g < G; ++g)
      if (cbase + g < ncol && !st[cbase + g].done) any = true;
    if (!any) return;
  }
  extern __shared__ double sm[];
  double *yr = sm;           // G x W row products
  double *rp = sm + G * W;   // G x W gathered right-hand sides (zero padded)
  double *yc = rp;           // after the rows: NW waves x G x W column products
  const int64_t p = chunk_patch[blockIdx.x];
  const int r0 = chunk_rows[2 * blockIdx.x], r1 = chunk_rows[2 * blockIdx.x + 1];
  const int64_t c0 = patch_col[p];
  const int m = int(patch_col[p + 1] - c0);
  const int mS = (m + V - 1) / V * V;
  const T *A = inv + inv_off[p];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slot = lane / L, t = lane % L;
  auto load_row = [&](int i, bool ok, vecV *buf) {
    const int si = i / V * V;
    const T *row = A + seg_row_off(i, mS, V) - si;  // row[c] = stored entry of column c
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int c = q * V * L + t * V;
      if (ok && c >= si && c < mS)
        buf[q] = NT ? __builtin_nontemporal_load(reinterpret_cast<const vecV *>(row + c))
                    : *reinterpret_cast<const vecV *>(row + c);
      else buf[q] = vecV(0);
    }
  };
  // rows in flight: a ring of D row buffers, D - 1 loads ahead of the
  // products; the first loads are issued before the gather of the patch
  // right-hand sides
  const int step = NW * RPW;
  const int niter = (r1 - r0 + step - 1) / step;
  const int i0 = r0 + wave * RPW + slot;
  vecV buf[D][NQ];
#pragma unroll
  for (int u = 0; u < D - 1; ++u) load_row(i0 + u * step, i0 + u * step < r1, buf[u]);
  for (int t2 = threadIdx.x; t2 < G * W; t2 += 64 * NW) {
    const int g = t2 / W, j = t2 - g * W;
    double sv = 0;
    if (j < m && cbase + g < ncol) {
      const double *rc = r + int64_t(cbase + g) * ldr;
      for (int64_t e = col_ent[c0 + j]; e < col_ent[c0 + j + 1]; ++e) sv += ent_coef[e] * rc[ent_dof[e]];
    }
    rp[t2] = sv;
    yr[t2] = 0.0;
  }
  __syncthreads();
  C rj[NQ][G][V], cacc[NQ][G][V];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int h = 0; h < V; ++h) {
        rj[q][g][h] = C(rp[g * W + q * V * L + t * V + h]);
        cacc[q][g][h] = C(0);
      }
  for (int it = 0; it < niter; it += D) {
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int k = it + u;
      if (k >= niter) break;  // uniform over the block
      const int i = i0 + k * step;
      const int ia = i + (D - 1) * step;
      load_row(ia, ia < r1, buf[(u + D - 1) % D]);
      const bool ok = i < r1;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const C ri = ok ? C(rp[g * W + i]) : C(0);
        C rs = C(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int h = 0; h < V; ++h) {
            const C a = widen(buf[u][q][h]);
            rs += a * rj[q][g][h];
            cacc[q][g][h] += a * ri;
          }
        rs = group_sum<L>(rs);
        if (ok && t == 0) yr[g * W + i] = double(rs);
      }
    }
  }
  // column products: sum the row slots of the wave, then one LDS row per wave
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int h = 0; h < V; ++h) {
        C v = cacc[q][g][h];
        if (L <= 16) v += __shfl_xor(v, 16, 64);
        if (L <= 32) v += __shfl_xor(v, 32, 64);
        cacc[q][g][h] = v;
      }
  __syncthreads();  // the column products overwrite the right-hand sides
  if (slot == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int h = 0; h < V; ++h) yc[(wave * G + g) * W + q * V * L + t * V + h] = double(cacc[q][g][h]);
  }
  __syncthreads();
  for (int t2 = threadIdx.x; t2 < G * m; t2 += 64 * NW) {
    const int g = t2 / m, j = t2 - g * m;
    if (j < r0 || cbase + g >= ncol) continue;
    double cs = yc[g * W + j];
    if (NW == 4)
      cs = (cs + yc[(1 * G + g) * W + j]) + (yc[(2 * G + g) * W + j] + yc[(3 * G + g) * W + j]);
    const double y = scale * (yr[g * W + j] + cs);
    double *zc = z + int64_t(cbase + g) * ldz;
    for (int64_t e = col_ent[c0 + j]; e < col_ent[c0 + j + 1]; ++e) atomicAdd(&zc[ent_dof[e]], ent_coef[e] * y);
  }
}

// Patch solves from the folded layout (see kFoldMin): a chunk of pair rows
// k in [k0, k1) of one patch, G right-hand sides (blockIdx.y).  A wave works
// on 64 / L pair rows at a time, L lanes each; lane t owns positions
// p = q V L + t V + [0, V), q < NQ, of both halves, i.e. the fixed columns p
// (first half, p < h) and h + p (second half, and the trailing block's rows
// in the first half).  Per entry, with a = first-half entry and b =
// second-half entry of pair row k:
//   p >= k: a = A[k][p]:          y_k += a r_p,     y_p += a r_k
//   p <  k: a = A[h+p][h+k-1]:    y_{h+k-1} += a r_{h+p},  y_{h+p} += a r_{h+k-1}
//           b = A[k][h+p]:        y_k += b r_{h+p}, y_{h+p} += b r_k
// The two row sums of a pair row are summed over its L lanes (DPP); the
// column products stay in registers until the end of the chunk.  Every load
// slot below hP carries an entry.
#ifndef RZ_FOLD_RL
#define RZ_FOLD_RL 8
#endif
template <int V, int L, int NQ, int G, int D, typename T, int NW, bool NT>
__global__ __launch_bounds__(64 * NW) void k_patch_fold(const int64_t *__restrict__ chunk_patch,
                                                    const int32_t *__restrict__ chunk_rows,
                                                    const int64_t *__restrict__ patch_col,
                                                    const int64_t *__restrict__ col_ent,
                                                    const int32_t *__restrict__ ent_dof,
                                                    const double *__restrict__ ent_coef,
                                                    const int64_t *__restrict__ inv_off, const T *__restrict__ inv,
                                                    const double *__restrict__ r, int64_t ldr, double *__restrict__ z,
                                                    int64_t ldz, int ncol, double scale, const PcgState *st) {
  typedef decltype(widen(T())) C;
  constexpr int RPW = 64 / L;        // pair rows per wave step
  constexpr int W = NQ * L * V;      // positions of a half (>= hP)
  constexpr int W2 = 2 * W;          // LDS stride: patch dofs 0 .. 2W - 1
  typedef T vecV __attribute__((ext_vector_type(V)));
  const int cbase = blockIdx.y * G;
  if (st) {
    bool any = false;
    for (int g = 0; g < G; ++g)
      if (cbase + g < ncol && !st[cbase + g].done) any = true;
    if (!any) return;
  }
  extern __shared__ double sm[];
  double *yr = sm;            // G x W2 row products
  double *rp = sm + G * W2;   // G x W2 gathered right-hand sides (zero padded)
  double *yc = rp;            // after the rows: NW waves x G x W2 column products
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slot = lane / L, t = lane % L;
  const int64_t pt = chunk_patch[blockIdx.x];
  const int k0 = chunk_rows[2 * blockIdx.x], k1 = chunk_rows[2 * blockIdx.x + 1];
  const int64_t c0 = patch_col[pt];
  const int m = int(patch_col[pt + 1] - c0);
  const int h = (m + 1) >> 1, hP = fold_hp(m, int(sizeof(T)));
  const T *A = inv + inv_off[pt];
  auto load_row = [&](int k, bool ok, vecV *b1, vecV *b2) {
    const T *row = A + int64_t(k) * 2 * hP;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int c = q * V * L + t * V;
      if (ok && c < hP) {
        b1[q] = NT ? __builtin_nontemporal_load(reinterpret_cast<const vecV *>(row + c))
                   : *reinterpret_cast<const vecV *>(row + c);
        b2[q] = NT ? __builtin_nontemporal_load(reinterpret_cast<const vecV *>(row + hP + c))
                   : *reinterpret_cast<const vecV *>(row + hP + c);
      } else {
        b1[q] = vecV(0);
        b2[q] = vecV(0);
      }
    }
  };
  // pair rows in flight: a ring of D buffers, D - 1 loads ahead of the
  // products (with one buffer, the first row's load); the first loads are
  // issued before the gather of the right-hand sides
  const int step = NW * RPW;
  const int niter = (k1 - k0 + step - 1) / step;
  const int i0 = k0 + wave * RPW + slot;
  constexpr int D0 = D == 1 ? 1 : D - 1;
  vecV buf[D][2][NQ];
#pragma unroll
  for (int u = 0; u < D0; ++u) load_row(i0 + u * step, i0 + u * step < k1, buf[u][0], buf[u][1]);
  for (int t2 = threadIdx.x; t2 < G * W2; t2 += 64 * NW) {
    const int g = t2 / W2, j = t2 - g * W2;
    double sv = 0;
    if (j < m && cbase + g < ncol) {
      const double *rc = r + int64_t(cbase + g) * ldr;
      for (int64_t e = col_ent[c0 + j]; e < col_ent[c0 + j + 1]; ++e) sv += ent_coef[e] * rc[ent_dof[e]];
    }
    rp[t2] = sv;
    yr[t2] = 0.0;
  }
  __syncthreads();
  // the right-hand side values of the lane's columns: registers, or for
  // FP64 entries with NQ V >= RZ_FOLD_RL LDS reads per pair row (fewer
  // registers, more waves per SIMD: measured 2-5% faster on the 431-855-dof
  // star sets).  Reduced-precision entries keep them in registers: an LDS
  // read per entry would move 4-8 times the streamed bytes through LDS.
  constexpr bool RL = sizeof(T) == 8 && NQ * V >= RZ_FOLD_RL;
  C rA[RL ? 1 : NQ][G][V], rB[RL ? 1 : NQ][G][V], accA[NQ][G][V], accB[NQ][G][V];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int c = q * V * L + t * V + v;
        if (!RL) {
          rA[q][g][v] = C(rp[g * W2 + c]);
          rB[q][g][v] = C(rp[g * W2 + h + c]);
        }
        accA[q][g][v] = C(0);
        accB[q][g][v] = C(0);
      }
  for (int it = 0; it < niter; it += D) {
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int kk = it + u;
      if (kk >= niter) break;  // uniform over the block
      const int k = i0 + kk * step;
      const int ka = k + (D - 1) * step;
      if (D > 1 || kk > 0) load_row(ka, ka < k1, buf[(u + D - 1) % D][0], buf[(u + D - 1) % D][1]);
      const bool ok = k < k1;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const C rk = ok ? C(rp[g * W2 + k]) : C(0);
        const C rk2 = (ok && k >= 1) ? C(rp[g * W2 + h + k - 1]) : C(0);
        C s1 = C(0), s2 = C(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const C a = widen(buf[u][0][q][v]), b = widen(buf[u][1][q][v]);
            const int c = q * V * L + t * V + v;
            const C ra = RL ? C(rp[g * W2 + c]) : rA[RL ? 0 : q][g][v];
            const C rb = RL ? C(rp[g * W2 + h + c]) : rB[RL ? 0 : q][g][v];
            const bool up = c >= k;
            const C a1 = up ? a : C(0), a2 = up ? C(0) : a;
            s1 += a1 * ra + b * rb;
            s2 += a2 * rb;
            accA[q][g][v] += a1 * rk;
            accB[q][g][v] += b * rk + a2 * rk2;
          }
        s1 = group_sum<L>(s1);
        s2 = group_sum<L>(s2);
        if (ok && t == 0) {
          if (k < h) yr[g * W2 + k] = double(s1);
          if (k >= 1) yr[g * W2 + h + k - 1] = double(s2);
        }
      }
    }
  }
  // column products: sum the pair-row slots of the wave, then one LDS row
  // per wave (first-half positions below h, and every second-half one)
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int v = 0; v < V; ++v) {
        C a = accA[q][g][v], b = accB[q][g][v];
        if (L <= 16) a += __shfl_xor(a, 16, 64), b += __shfl_xor(b, 16, 64);
        if (L <= 32) a += __shfl_xor(a, 32, 64), b += __shfl_xor(b, 32, 64);
        accA[q][g][v] = a;
        accB[q][g][v] = b;
      }
  __syncthreads();  // the column products overwrite the right-hand sides
  if (slot == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const int c = q * V * L + t * V + v;
          double *row = yc + (wave * G + g) * W2;
          if (c < h) row[c] = double(accA[q][g][v]);
          row[h + c] = double(accB[q][g][v]);
        }
  }
  __syncthreads();
  for (int t2 = threadIdx.x; t2 < G * m; t2 += 64 * NW) {
    const int g = t2 / m, j = t2 - g * m;
    if ((j < h && j < k0) || cbase + g >= ncol) continue;
    double cs = yc[g * W2 + j];
    if (NW == 4)
      cs = (cs + yc[(1 * G + g) * W2 + j]) + (yc[(2 * G + g) * W2 + j] + yc[(3 * G + g) * W2 + j]);
    const double y = scale * (yr[g * W2 + j] + cs);
    double *zc = z + int64_t(cbase + g) * ldz;
    for (int64_t e = col_ent[c0 + j]; e < col_ent[c0 + j + 1]; ++e) atomicAdd(&zc[ent_dof[e]], ent_coef[e] * y);
  }
}

// Reduced-precision copy of a patch inverse: from the V = 2 FP64 segmented
// layout to the VT-element layout of T (VT = 16 bytes / sizeof(T))
template <typename T, int VT>
__global__ void k_seg_to_low(const int64_t *__restrict__ patch_col, const int64_t *__restrict__ off64,
                             const int64_t *__restrict__ offlo, const double *__restrict__ A, T *__restrict__ B) {
  const int64_t p = blockIdx.x;
  const int m = int(patch_col[p + 1] - patch_col[p]);
  const int m2 = (m + 1) / 2 * 2, mv = (m + VT - 1) / VT * VT;
  const double *a = A + off64[p];
  T *b = B + offlo[p];
  for (int i = 0; i < m; ++i) {
    const int s2 = i / 2 * 2, sv = i / VT * VT;
    const double *ra = a + seg_row_off(i, m2, 2) - s2;
    T *rb = b + seg_row_off(i, mv, VT) - sv;
    for (int c = sv + threadIdx.x; c < mv; c += blockDim.x) rb[c] = from_f64<T>((c >= i && c < m) ? ra[c] : 0.0);
  }
}

// Reduced-precision copy of a folded patch inverse: the halves of the pair
// rows change length from the FP64 hP to that of T (zero padded)
template <typename T, int VT>
__global__ void k_fold_to_low(const int64_t *__restrict__ patch_col, const int64_t *__restrict__ off64,
                              const int64_t *__restrict__ offlo, const double *__restrict__ A, T *__restrict__ B) {
  const int64_t p = blockIdx.x;
  const int m = int(patch_col[p + 1] - patch_col[p]);
  const int h = (m + 1) / 2, h2 = fold_hp(m, 8), hv = fold_hp(m, int(sizeof(T)));
  const double *a = A + off64[p];
  T *b = B + offlo[p];
  const int64_t total = int64_t(h + 1) * 2 * hv;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int64_t k = e / (2 * hv);
    const int q = int(e % (2 * hv)), half = q / hv, c = q % hv;
    b[e] = from_f64<T>(c < h2 ? a[k * 2 * h2 + half * h2 + c] : 0.0);
  }
}

// Coarse solve zW += A_W^{-1} rW with the inverse as packed upper 64 x 64
// tiles (I <= J; diagonal tiles full).  A block takes tiles J in [J0, J1) of
// tile row I, G right-hand sides: thread (c, ty) holds rows 16 ty .. 16 ty + 15
// of column c of the tile.  Row products A_IJ rW_J stay in registers for the
// whole strip (one lane reduction at the end); column products A_IJ^T rW_I
// are summed over the four waves in LDS and added to zW_J per tile.
template <int G, typename T, bool NTL>
__global__ __launch_bounds__(256) void k_coarse_symv(int NT, int S, const T *__restrict__ tiles,
                                                     const double *__restrict__ rW, double *__restrict__ zW,
                                                     int npad, int ncol, const PcgState *st) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const int I = blockIdx.x;
  const int J0 = max(I, int(blockIdx.y) * S), J1 = min(NT, int(blockIdx.y + 1) * S);
  if (J0 >= J1) return;
  const int cbase = blockIdx.z * G;
  if (st) {
    bool any = false;
    for (int g = 0; g < G; ++g)
      if (cbase + g < ncol && !st[cbase + g].done) any = true;
    if (!any) return;
  }
  __shared__ double cl[2][G][4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  double rI[G][16], acc[G][16];
  const double *rc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    rc[g] = rW + int64_t(min(cbase + g, ncol - 1)) * npad;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      rI[g][k] = cbase + g < ncol ? rc[g][I * 64 + ty * 16 + k] : 0.0;
      acc[g][k] = 0.0;
    }
  }
  const T *row = tiles + (int64_t(I) * NT - int64_t(I) * (I - 1) / 2 - I) * 4096 + ty * 1024 + tx * 2;
  auto load = [&](int J, v2 *buf) {
    const T *tp = row + int64_t(J) * 4096;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      buf[q] = NTL ? __builtin_nontemporal_load(reinterpret_cast<const v2 *>(tp + q * 128))
                   : *reinterpret_cast<const v2 *>(tp + q * 128);
  };
  v2 cur[8], nxt[8];
  load(J0, cur);
  int pb = 0;
  for (int J = J0; J < J1; ++J) {
    if (J + 1 < J1) load(J + 1, nxt);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const double rJ = rc[g][J * 64 + tx];
      double colp = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double a0 = to_f64(cur[q].x), a1 = to_f64(cur[q].y);
        acc[g][2 * q] += a0 * rJ;
        acc[g][2 * q + 1] += a1 * rJ;
        colp += a0 * rI[g][2 * q] + a1 * rI[g][2 * q + 1];
      }
      cl[pb][g][ty][tx] = colp;
    }
    __syncthreads();
    if (J > I && ty == 0) {
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (cbase + g < ncol)
          atomicAdd(&zW[int64_t(cbase + g) * npad + J * 64 + tx],
                    (cl[pb][g][0][tx] + cl[pb][g][1][tx]) + (cl[pb][g][2][tx] + cl[pb][g][3][tx]));
    }
    pb ^= 1;
#pragma unroll
    for (int q = 0; q < 8; ++q) cur[q] = nxt[q];
  }
  // row products: sum over the 64 columns (lanes); lane k keeps row 16 ty + k
#pragma unroll
  for (int g = 0; g < G; ++g) {
    double mine = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const double v = group_sum<64>(acc[g][k]);
      if (tx == k) mine = v;
    }
    if (tx < 16 && cbase + g < ncol) atomicAdd(&zW[int64_t(cbase + g) * npad + I * 64 + ty * 16 + tx], mine);
  }
}

// ---- many columns: the coarse and small-patch solves as FP64 MFMA GEMMs
// Full coarse inverse in MFMA fragment order, built from the packed upper
// tiles: index (((I NT + J) 4 + w) 16 + kb) 64 + lane holds
// A[64 I + 16 w + lane % 16][64 J + 4 kb + lane / 16].
__global__ void k_coarse_expand(int NT, const double *__restrict__ T, double *__restrict__ F) {
  const int I = blockIdx.x, J = blockIdx.y;
  double *out = F + (int64_t(I) * NT + J) * 4096;
  for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
    const int lane = e & 63, kb = (e >> 6) & 15, w = e >> 10;
    const int r = 16 * w + (lane & 15), c = 4 * kb + (lane >> 4);
    double v;
    if (I <= J) {
      const int64_t t = int64_t(I) * NT - int64_t(I) * (I - 1) / 2 + (J - I);
      v = T[t * 4096 + ctile_idx(r, c)];
    } else {
      const int64_t t = int64_t(J) * NT - int64_t(J) * (J - 1) / 2 + (I - J);
      v = T[t * 4096 + ctile_idx(c, r)];
    }
    out[e] = v;
  }
}

// zW[64 I : 64 I + 64, 64 cg : 64 cg + 64] += sum_{J in split} A_IJ rW_J.
// Wave w owns rows 16 w .. 16 w + 15 of the block row; rW_J is staged in LDS
// (the next one is loaded into registers during the current MFMAs).
__global__ __launch_bounds__(256) void k_coarse_gemm(int NT, int nsplit, const double *__restrict__ F,
                                                     const double *__restrict__ rW, double *__restrict__ zW,
                                                     int npad, int ncol, const PcgState *st) {
  const int I = blockIdx.x, cg = blockIdx.y, sp = blockIdx.z;
  const int c0 = cg * 64;
  if (st) {
    bool any = false;
    for (int c = c0; c < min(ncol, c0 + 64); ++c)
      if (!st[c].done) any = true;
    if (!any) return;
  }
  __shared__ double R[64][65];  // R[k][col]
  const int J0 = int(int64_t(NT) * sp / nsplit), J1 = int(int64_t(NT) * (sp + 1) / nsplit);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  d4 acc[4];
  for (int nb = 0; nb < 4; ++nb) acc[nb] = d4{0, 0, 0, 0};
  // thread t stages 16 entries: column (t / 4), rows 16 (t % 4) .. + 15
  const int scol = threadIdx.x >> 2, srow = (threadIdx.x & 3) * 16;
  double stage[16];
  auto load_R = [&](int J) {
    const int c = c0 + scol;
    const double *src = rW + int64_t(c) * npad + int64_t(J) * 64 + srow;
#pragma unroll
    for (int e = 0; e < 16; ++e) stage[e] = c < ncol ? src[e] : 0.0;
  };
  // the wave's 16 A fragments of tile J, loaded one tile ahead (a load's
  // latency spans several tiles' MFMA time at this occupancy)
  double a[16];
  auto load_A = [&](int J) {
    const double *Af = F + ((int64_t(I) * NT + J) * 4 + wave) * 1024 + lane;
#pragma unroll
    for (int kb = 0; kb < 16; ++kb) a[kb] = Af[kb * 64];
  };
  if (J0 < J1) {
    load_R(J0);
    load_A(J0);
  }
  for (int J = J0; J < J1; ++J) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) R[srow + e][scol] = stage[e];
    __syncthreads();
    double ac[16];
#pragma unroll
    for (int kb = 0; kb < 16; ++kb) ac[kb] = a[kb];
    if (J + 1 < J1) {
      load_R(J + 1);
      load_A(J + 1);
    }
#pragma unroll
    for (int kb = 0; kb < 16; ++kb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[kb], R[kb * 4 + lk][nb * 16 + li], acc[nb], 0, 0, 0);
  }
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int c = c0 + nb * 16 + li;
    if (c >= ncol) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = I * 64 + wave * 16 + lk + 4 * v;
      atomicAdd(&zW[int64_t(c) * npad + row], acc[nb][v]);
    }
  }
}

// ---- multi-column patch solves on MFMA (sets of patches up to kFoldMin
// dofs, 8 or more columns).  Each patch inverse is copied once into MFMA
// A-fragment order (full MP x MP, zero padded); per block one patch and up
// to 64 columns: the gathered right-hand sides are staged in LDS as B
// fragments, one wave per 16-row block computes Z_p = A_p R_p for the four
// 16-column blocks, and Z_p goes to a buffer indexed by patch column;
// k_patch_zb_scatter then adds each dof's entries in a fixed order
// (deterministic, no atomics).  The right-hand sides of the set's dofs are
// first copied dof-major (k_patch_rt: rt[a * NC + c], NC the buffer's
// columns) and the results are written dof-major too (zb[pr * NC + c]):
// with the column-major vectors (columns 8 MB apart) each block touched
// some 200 pages and the address translation thrashed.
//   FP64 (mfma_f64_16x16x4f64): MP = m rounded up to 16; fragment (mb, kb)
//     lane l = A[16 mb + l % 16][4 kb + l / 16]; B lane l = R[4 kb + l / 16]
//     [16 nb + l % 16]; accumulator v = Z[16 mb + l / 16 + 4 v][16 nb + l % 16].
//   bfloat16 (mfma_f32_16x16x32_bf16, FP32 accumulation): MP = m rounded up
//     to 32; fragment (mb, kb) lane l, element j = A[16 mb + l % 16]
//     [32 kb + 8 (l / 16) + j]; B likewise R[32 kb + 8 (l / 16) + j][16 nb +
//     l % 16]; accumulator v = Z[16 mb + 4 (l / 16) + v][16 nb + l % 16].
//     The right-hand sides are split r = r_hi + r_lo into two bfloat16 parts
//     (their sum carries 16 significant bits) and both are multiplied, so
//     the patch solve applies the bfloat16-stored inverse to r with FP32
//     accumulation like the streamed kernels do.
//   FP32 (mfma_f32_16x16x4f32, the FP32 copies of RZ_FP32_PC / RZ_FP32_IR):
//     the FP64 fragment and B layouts with FP32 values (r rounded to FP32,
//     of the order of the inverse's own rounding); accumulator v = Z[16 mb +
//     4 (l / 16) + v][16 nb + l % 16] as for bfloat16.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename F>
struct FragTraits;
template <>
struct FragTraits<double> {
  static constexpr int KS = 4, MPA = 16;  // k per MFMA, padding of MP
  typedef double A_t;
  typedef double Z_t;
};
template <>
struct FragTraits<uint16_t> {
  static constexpr int KS = 32, MPA = 32;
  typedef uint4 A_t;   // 8 bfloat16 bits
  typedef float Z_t;
};
template <>
struct FragTraits<float> {  // mfma_f32_16x16x4f32: the FP64 operand layouts
  static constexpr int KS = 4, MPA = 16;
  typedef float A_t;
  typedef float Z_t;
};

__device__ inline uint16_t bf16_bits(float v) {  // round to nearest even
  uint32_t u = __float_as_uint(v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

template <typename F>
__global__ void k_seg_to_frag(const int64_t *__restrict__ patch_col, const int64_t *__restrict__ seg_off,
                              const double *__restrict__ P, const int64_t *__restrict__ frag_off,
                              F *__restrict__ out) {
  constexpr int KS = FragTraits<F>::KS, MPA = FragTraits<F>::MPA;
  const int64_t p = blockIdx.x;
  const int m = int(patch_col[p + 1] - patch_col[p]);
  const int MP = (m + MPA - 1) / MPA * MPA, KB = MP / KS, mS = (m + 1) / 2 * 2;
  const double *S = P + seg_off[p];
  F *o = out + frag_off[p];
  const int64_t total = int64_t(MP) * MP;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    int i, k;
    if constexpr (KS == 4) {  // e = (mb KB + kb) 64 + l
      const int l = int(e & 63), blk = int(e >> 6);
      i = 16 * (blk / KB) + (l & 15);
      k = 4 * (blk % KB) + (l >> 4);
    } else {                  // e = ((mb KB + kb) 64 + l) 8 + j
      const int j = int(e & 7), l = int((e >> 3) & 63), blk = int(e >> 9);
      i = 16 * (blk / KB) + (l & 15);
      k = 32 * (blk % KB) + 8 * (l >> 4) + j;
    }
    double v = 0.0;
    if (i < m && k < m) {
      const int a = min(i, k), b = max(i, k);
      v = (a == b ? 2.0 : 1.0) * S[seg_row_off(a, mS, 2) + b - a / 2 * 2];
    }
    if constexpr (KS == 4) o[e] = F(v);
    else o[e] = bf16_bits(float(v));
  }
}

// rt[a * NC + c] = r[c * ldr + adof[a]] for the set's dofs a and columns
// c < ncol: a 64-dof x 64-column tile per block through LDS (reads along
// columns, writes along dof rows)
__global__ __launch_bounds__(256) void k_patch_rt(int64_t na, const int32_t *__restrict__ adof,
                                                  const double *__restrict__ r, int64_t ldr, int ncol,
                                                  double *__restrict__ rt, int NC) {
  __shared__ double tile[64][65];
  const int64_t a0 = int64_t(blockIdx.x) * 64;
  const int c0 = blockIdx.y * 64;
  const int t = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t a = a0 + t;
  const int32_t d = a < na ? adof[a] : 0;
  for (int c = w; c < 64; c += 4)
    tile[c][t] = (a < na && c0 + c < ncol) ? r[int64_t(c0 + c) * ldr + d] : 0.0;
  __syncthreads();
  for (int i = w; i < 64; i += 4)
    if (a0 + i < na && c0 + t < ncol) rt[(a0 + i) * NC + c0 + t] = tile[t][i];
}

template <typename F, int MPMAX>
__global__ __launch_bounds__(64 * (MPMAX / 16)) void k_patch_mfma(
    const int64_t *__restrict__ patch_col, const int64_t *__restrict__ col_ent, const int32_t *__restrict__ ent_a,
    const double *__restrict__ ent_coef, const int64_t *__restrict__ frag_off, const F *__restrict__ frag,
    const double *__restrict__ rt, typename FragTraits<F>::Z_t *__restrict__ zb, int NC, int ncol,
    const PcgState *st) {
  constexpr int KS = FragTraits<F>::KS, MPA = FragTraits<F>::MPA;
  constexpr bool BF = KS == 32;
  constexpr bool F32 = std::is_same<F, float>::value;
  typedef typename FragTraits<F>::A_t A_t;
  typedef typename FragTraits<F>::Z_t Z_t;
  typedef Z_t acc_t __attribute__((ext_vector_type(4)));
  const int64_t p = blockIdx.x;
  const int c0 = blockIdx.y * 64;
  if (st) {
    bool any = false;
    for (int c = c0; c < min(ncol, c0 + 64); ++c)
      if (!st[c].done) any = true;
    if (!any) return;
  }
  // B fragments in LDS, in units U (FP64: one double; bfloat16: 8 halves):
  // fragment (kb, nb) lane l at (kb 4 + nb) 68 + 17 (l / 16) + l % 16 -- each
  // 16-lane group padded by one unit, so the gather's writes (lanes apart by
  // one row k) fall in different banks; the bfloat16 lo parts follow the hi
  // parts at KB 4 68 units
  extern __shared__ double sm[];
  double *Rd = sm;
  float *Rf = reinterpret_cast<float *>(sm);
  uint4 *Ru = reinterpret_cast<uint4 *>(sm);
  uint16_t *Rh = reinterpret_cast<uint16_t *>(sm);
  const int64_t cb = patch_col[p];
  const int m = int(patch_col[p + 1] - cb);
  const int MP = (m + MPA - 1) / MPA * MPA, KB = MP / KS;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int mb = wave;
  const bool active = 16 * mb < MP;
  // the wave's A fragments, loaded before the gather (they do not depend on it)
  constexpr int KBMAX = MPMAX / KS;
  A_t a[KBMAX];
  if (active) {
    const A_t *Af = reinterpret_cast<const A_t *>(frag + frag_off[p]) + int64_t(mb) * KB * 64 + lane;
#pragma unroll
    for (int kb = 0; kb < KBMAX; ++kb)
      if (kb < KB) a[kb] = Af[kb * 64];
  }
  // gather of the right-hand sides into the B fragments
  if constexpr (!BF && !F32) {
    // FP64: thread t takes patch column k = t % MP and the 16 columns of
    // group t / MP (4 MP = the block's threads), its map entries loaded once
    // and the 16 right-hand side values read as one dof-major row piece (at
    // the occupancy the FP64 A fragments leave, one map chain per thread
    // beats the coalesced form below)
    const int t = threadIdx.x;
    const int k = t % MP, cg = t / MP;
    if (cg < 4) {
      double v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = 0.0;
      if (k < m)
        for (int64_t e = col_ent[cb + k]; e < col_ent[cb + k + 1]; ++e) {
          const double *row = rt + int64_t(ent_a[e]) * NC + c0 + 16 * cg;
          const double cf = ent_coef[e];
#pragma unroll
          for (int j = 0; j < 16; ++j)
            if (c0 + 16 * cg + j < ncol) v[j] += cf * row[j];
        }
      double *dst = Rd + ((k >> 2) * 4 + cg) * 68 + (k & 3) * 17;
#pragma unroll
      for (int j = 0; j < 16; ++j) dst[j] = v[j];
    }
  } else {
    // FP32 and bfloat16: 16 lanes take 16 consecutive columns of one patch
    // row k (the row's four column groups on the wave's four 16-lane groups:
    // one 512-byte piece of a dof-major row of rt per wave and map entry);
    // the block's MPMAX / 4 lane groups step over the MP x 4 (row, group)
    // pairs
    const int cl = threadIdx.x & 15;
    for (int q = threadIdx.x >> 4; q < 4 * MP; q += MPMAX / 4) {
      const int k = q >> 2, cg = q & 3;
      const int c = c0 + 16 * cg + cl;
      double v = 0.0;
      if (k < m && c < ncol)
        for (int64_t e = col_ent[cb + k]; e < col_ent[cb + k + 1]; ++e)
          v += ent_coef[e] * rt[int64_t(ent_a[e]) * NC + c];
      if constexpr (F32) {
        Rf[((k >> 2) * 4 + cg) * 68 + (k & 3) * 17 + cl] = float(v);
      } else {
        const int kb = k >> 5, kk = k & 31;
        const int u = ((kb * 4 + cg) * 68 + (kk >> 3) * 17) * 8 + (kk & 7) + 8 * cl;
        const float vf = float(v);
        const uint16_t hi = bf16_bits(vf);
        Rh[u] = hi;
        Rh[KB * 4 * 68 * 8 + u] = bf16_bits(vf - __uint_as_float(uint32_t(hi) << 16));
      }
    }
  }
  __syncthreads();
  if (!active) return;
  acc_t acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = acc_t{0, 0, 0, 0};
  const int lu = (lane >> 4) * 17 + (lane & 15);
#pragma unroll
  for (int kb = 0; kb < KBMAX; ++kb) {
    // a guarded body, not a break: the loop then unrolls fully and a[] stays
    // in registers (with the early exit the FP64 instances above 64 dofs
    // kept a[] in scratch, each fragment load waiting for its store)
    if (kb < KB)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      if constexpr (F32) {
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kb], Rf[(kb * 4 + nb) * 68 + lu], acc[nb], 0, 0, 0);
      } else if constexpr (!BF) {
        acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kb], Rd[(kb * 4 + nb) * 68 + lu], acc[nb], 0, 0, 0);
      } else {
        const int u = (kb * 4 + nb) * 68 + lu;
        const bf16x8 av = __builtin_bit_cast(bf16x8, a[kb]);
        const bf16x8 bh = __builtin_bit_cast(bf16x8, Ru[u]);
        const bf16x8 bl = __builtin_bit_cast(bf16x8, Ru[KB * 4 * 68 + u]);
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bh, acc[nb], 0, 0, 0);
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bl, acc[nb], 0, 0, 0);
      }
    }
  }
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int c = c0 + nb * 16 + li;
    if (c >= ncol) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * mb + ((BF || F32) ? 4 * lk + v : lk + 4 * v);
      if (row < m) zb[(cb + row) * NC + c] = acc[nb][v];
    }
  }
}

// z[c][d] += scale sum_e coef_e zb[pr_e * NC + c] over the dofs d of a
// patch set (ascending), entries in a fixed order: a 64-dof x 64-column
// tile per block, the dof sums staged in LDS as tile[column][dof], then
// added to z along columns.  FP64 entries: a wave sums one dof at a time
// with its lanes along the 64 columns (one coalesced 512-byte piece of a zb
// row per entry).  FP32 entries: a thread sums one dof over 16 columns
// (one 64-byte row piece per entry; with half the bytes per entry the
// dependent map loads of the coalesced form cost more than they save).
template <typename Z>
__global__ __launch_bounds__(256) void k_patch_zb_scatter(int64_t nd, const int32_t *__restrict__ dof,
                                                          const int64_t *__restrict__ ptr,
                                                          const int32_t *__restrict__ pr,
                                                          const double *__restrict__ coef,
                                                          const Z *__restrict__ zb, int NC,
                                                          double *__restrict__ z, int64_t ldz, int ncol,
                                                          double scale, const PcgState *st) {
  __shared__ double tile[64][65];
  const int64_t a0 = int64_t(blockIdx.x) * 64;
  const int c0 = blockIdx.y * 64;
  const int t = threadIdx.x & 63, w = threadIdx.x >> 6;
  if constexpr (sizeof(Z) == 8) {
    const int c = c0 + t;
#pragma unroll 4
    for (int i = w; i < 64; i += 4) {
      const int64_t a = a0 + i;
      double v = 0.0;
      if (a < nd && c < ncol)
        for (int64_t e = ptr[a]; e < ptr[a + 1]; ++e) v += coef[e] * double(zb[int64_t(pr[e]) * NC + c]);
      tile[t][i] = v;
    }
  } else {
    const int64_t a = a0 + t;
    double v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = 0.0;
    if (a < nd)
      for (int64_t e = ptr[a]; e < ptr[a + 1]; ++e) {
        const Z *row = zb + int64_t(pr[e]) * NC + c0 + 16 * w;
        const double cf = coef[e];
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (c0 + 16 * w + j < ncol) v[j] += cf * double(row[j]);
      }
#pragma unroll
    for (int j = 0; j < 16; ++j) tile[16 * w + j][t] = v[j];
  }
  __syncthreads();
  const int64_t a = a0 + t;
  if (a >= nd) return;
  const int64_t d = dof[a];
  for (int cc = w; cc < 64; cc += 4) {
    const int col = c0 + cc;
    if (col < ncol && !(st && st[col].done)) z[int64_t(col) * ldz + d] += scale * tile[cc][t];
  }
}

// -------------------------------------------------------------- Krylov
// Multi-column PCG: column c of every vector lives at base + c * ld; each
// column has its own state st[c] and RB block partials at part[c * RB ...].
// A reduction kernel leaves the partials; the kernel consuming the scalar
// re-sums them in every block (fixed order, all blocks agree bit for bit), so
// the kernel boundary makes them visible without device-scope fences.
__device__ inline double sum_part(const double *part, int RB, double *sm4) {
  double v = 0;
  for (int i = threadIdx.x; i < RB; i += 256) v += part[i];
  return block_sum256(v, sm4);
}

// coarse correction folded in: z_i + zW[t / N] when i = off + t, t % N == 0
__device__ inline double z_full(int64_t i, const double *z, const double *zW, const CoarseFold &cf) {
  double v = z[i];
  if (zW) {
    const int64_t t = i - cf.off;
    if (t >= 0 && t < cf.span && t % cf.N == 0) v += zW[t / cf.N];
  }
  return v;
}

__global__ __launch_bounds__(256) void k_dot_m(int64_t n, const double *__restrict__ a, int64_t lda,
                                               const double *__restrict__ b, int64_t ldb, CoarseFold cf, int npad,
                                               double *__restrict__ part, int RB, const PcgState *st) {
  const int c = blockIdx.y;
  if (st && st[c].done) return;
  __shared__ double sm4[4];
  const double *ac = a + c * lda, *bc = b + c * ldb;
  const double *zW = cf.zW ? cf.zW + int64_t(c) * npad : nullptr;
  double s = 0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(RB) * 256)
    s += ac[i] * z_full(i, bc, zW, cf);
  s = block_sum256(s, sm4);
  if (threadIdx.x == 0) part[c * RB + blockIdx.x] = s;
}

// PCG start: bb = ||b||^2, rr = ||r||^2 (partials in partZ / partR)
__global__ __launch_bounds__(256) void k_pcg_start(const double *__restrict__ partB, const double *__restrict__ partR,
                                                   int RB, double tol2, int maxit, PcgState *st,
                                                   const PcgState *outer) {
  __shared__ double sm4[4];
  const int c = blockIdx.x;
  const double bb = sum_part(partB + c * RB, RB, sm4);
  const double rr = sum_part(partR + c * RB, RB, sm4);
  if (threadIdx.x == 0) {
    PcgState &s = st[c];
    s.bb = bb;
    s.rr = rr;
    s.tol2 = tol2;
    s.iter = 0;
    s.maxit = maxit;
    s.status = PCG_RUNNING;
    s.done = 0;
    // columns already converged in an enclosing refinement loop are skipped
    if (!(bb > 0.0) || rr <= tol2 * bb || (outer && outer[c].done)) {
      s.done = 1;
      s.status = PCG_CONVERGED;
    }
  }
}

// alpha = rz / pAp; x += alpha p; r -= alpha Ap; partials of ||r||^2
__global__ __launch_bounds__(256) void k_update_xr_m(int64_t n, double *__restrict__ x, int64_t ldx,
                                                     double *__restrict__ r, const double *__restrict__ p,
                                                     const double *__restrict__ Ap, const double *__restrict__ partZ,
                                                     const double *__restrict__ partA, double *__restrict__ partR,
                                                     int RB, PcgState *st) {
  const int c = blockIdx.y;
  if (st[c].done) return;
  __shared__ double sm4[4];
  const double rz = sum_part(partZ + c * RB, RB, sm4);
  const double pAp = sum_part(partA + c * RB, RB, sm4);
  if (!(pAp > 0.0) || !isfinite(pAp) || !(rz > 0.0) || !isfinite(rz)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st[c].done = 1;
      st[c].status = PCG_BREAKDOWN;
    }
    return;
  }
  const double alpha = rz / pAp;
  double *xc = x + c * ldx, *rc = r + c * n;
  const double *pc = p + c * n, *apc = Ap + c * n;
  double s = 0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(RB) * 256) {
    xc[i] += alpha * pc[i];
    const double ri = rc[i] - alpha * apc[i];
    rc[i] = ri;
    s += ri * ri;
  }
  s = block_sum256(s, sm4);
  if (threadIdx.x == 0) {
    partR[c * RB + blockIdx.x] = s;
    if (blockIdx.x == 0) {
      st[c].rz = rz;
      st[c].pAp = pAp;
      st[c].alpha = alpha;
      if (st[c].iter < kMaxIter) st[c].alphas[st[c].iter] = alpha;
    }
  }
}

// convergence test on ||r||^2, then z = D_I^{-1} r (0 off the interior) and
// the coarse gather rW = R_W r, zW = 0 (all for column blockIdx.y)
__global__ __launch_bounds__(256) void k_check_jacobi_m(int64_t n, int64_t offI, const double *__restrict__ dinv,
                                                        const double *__restrict__ r, double *__restrict__ z,
                                                        int nW, int npad, const int32_t *__restrict__ wd,
                                                        double *__restrict__ rW, double *__restrict__ zW,
                                                        const double *__restrict__ partR, int RB, PcgState *st) {
  const int c = blockIdx.y;
  if (st[c].done) return;
  __shared__ double sm4[4];
  const double rr = sum_part(partR + c * RB, RB, sm4);
  const bool bad = !isfinite(rr), conv = rr <= st[c].tol2 * st[c].bb;  // identical in every block
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // only this thread reads and writes the iteration count
    const int it = st[c].iter + 1;
    st[c].rr = rr;
    st[c].iter = it;
    if (bad || conv || it >= st[c].maxit) {
      st[c].status = bad ? PCG_BREAKDOWN : (conv ? PCG_CONVERGED : PCG_MAXIT);
      st[c].done = 1;
    }
  }
  // at the iteration cap the remaining blocks still form z, which is then unused
  if (bad || conv) return;
  const double *rc = r + c * n;
  double *zc = z + c * n, *rWc = rW + int64_t(c) * npad, *zWc = zW + int64_t(c) * npad;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    zc[i] = i >= offI ? rc[i] * dinv[i - offI] : 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < npad; i += stride) {
    rWc[i] = i < nW ? rc[wd[i]] : 0.0;
    zWc[i] = 0.0;
  }
}

// beta = rz_new / rz; p = z + beta p (coarse part folded in); Ap = 0
__global__ __launch_bounds__(256) void k_update_p_m(int64_t n, double *__restrict__ p, const double *__restrict__ z,
                                                    CoarseFold cf, int npad, double *__restrict__ Ap,
                                                    const double *__restrict__ partZ, int RB, PcgState *st) {
  const int c = blockIdx.y;
  if (st[c].done) return;
  __shared__ double sm4[4];
  const double rz_new = sum_part(partZ + c * RB, RB, sm4);
  const double beta = rz_new / st[c].rz;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st[c].beta = beta;
    if (st[c].iter - 1 < kMaxIter) st[c].betas[st[c].iter - 1] = beta;
  }
  double *pc = p + c * n, *apc = Ap + c * n;
  const double *zc = z + c * n;
  const double *zW = cf.zW ? cf.zW + int64_t(c) * npad : nullptr;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    pc[i] = z_full(i, zc, zW, cf) + beta * pc[i];
    apc[i] = 0.0;
  }
}

// per column: r = b - Ax (b at ldb), p = 0 (set later), used at the start
__global__ void k_residual_m(int64_t n, const double *__restrict__ b, int64_t ldb, const double *__restrict__ Ax,
                             double *__restrict__ r) {
  const int c = blockIdx.y;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    r[c * n + i] = b[c * ldb + i] - Ax[c * n + i];
}

__global__ void k_fill_m(double *__restrict__ y, int64_t n, int64_t ld, const PcgState *st) {
  const int c = blockIdx.y;
  if (st && st[c].done) return;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[c * ld + i] = 0.0;
}

__global__ void k_copy_m(int64_t n, const double *__restrict__ a, int64_t lda, double *__restrict__ b, int64_t ldb) {
  const int c = blockIdx.y;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    b[c * ldb + i] = a[c * lda + i];
}

// coarse: rW = R_W r (all columns), zW = 0; and z += R_W^T zW
__global__ void k_coarse_gather_m(int nW, int npad, const int32_t *__restrict__ wd, const double *__restrict__ r,
                                  int64_t ldr, double *__restrict__ rW, double *__restrict__ zW,
                                  const uint8_t *__restrict__ dm) {
  const int c = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  rW[int64_t(c) * npad + i] = (i < nW && !(dm && dm[wd[i]])) ? r[c * ldr + wd[i]] : 0.0;
  zW[int64_t(c) * npad + i] = 0.0;
}

__global__ void k_coarse_scatter_m(int nW, int npad, const int32_t *__restrict__ wd, const double *__restrict__ zW,
                                   double *__restrict__ z, int64_t ldz) {
  const int c = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nW) z[c * ldz + wd[i]] += zW[int64_t(c) * npad + i];
}

__global__ void k_jacobi_m(int64_t n, int64_t offI, const double *__restrict__ dinv, const double *__restrict__ r,
                           int64_t ldr, double *__restrict__ z, int64_t ldz) {
  const int c = blockIdx.y;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    z[c * ldz + i] = i >= offI ? r[c * ldr + i] * dinv[i - offI] : 0.0;
}

// ---- symmetric multiplicative hybrid (Sec. 7.1): the sweep's small kernels
// First group of the sweep: z = rho_1^{-1} D_I^{-1} r on the interior, zero
// on the interface, and the tracked residual s = r.  With check set (inside
// PCG) it first takes the convergence test of k_check_jacobi_m.
__global__ __launch_bounds__(256) void k_hyb_init_m(int64_t n, int64_t offI, const double *__restrict__ dinv,
                                                    double w1, const double *__restrict__ r, int64_t ldr,
                                                    double *__restrict__ z, int64_t ldz, double *__restrict__ sres,
                                                    double *__restrict__ d, const double *__restrict__ partR, int RB,
                                                    PcgState *st) {
  const int c = blockIdx.y;
  if (st) {
    if (st[c].done) return;
    __shared__ double sm4[4];
    const double rr = sum_part(partR + c * RB, RB, sm4);
    const bool bad = !isfinite(rr), conv = rr <= st[c].tol2 * st[c].bb;  // identical in every block
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      const int it = st[c].iter + 1;
      st[c].rr = rr;
      st[c].iter = it;
      if (bad || conv || it >= st[c].maxit) {
        st[c].status = bad ? PCG_BREAKDOWN : (conv ? PCG_CONVERGED : PCG_MAXIT);
        st[c].done = 1;
      }
    }
    if (bad || conv) return;
  }
  const double *rc = r + c * ldr;
  double *zc = z + c * ldz, *sc = sres + c * n, *dc = d + c * n;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const double ri = rc[i];
    zc[i] = i >= offI ? w1 * ri * dinv[i - offI] : 0.0;
    sc[i] = ri;
    dc[i] = 0.0;
  }
}

// z += d (per column; columns that are done are skipped)
__global__ void k_add_m(int64_t n, const double *__restrict__ d, double *__restrict__ z, int64_t ldz,
                        const PcgState *st) {
  const int c = blockIdx.y;
  if (st && st[c].done) return;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    z[c * ldz + i] += d[c * n + i];
}

// last group of the sweep: z += rho_1^{-1} D_I^{-1} s on the interior
__global__ void k_jacobi_add_m(int64_t n, int64_t offI, const double *__restrict__ dinv, double w1,
                               const double *__restrict__ sres, double *__restrict__ z, int64_t ldz,
                               const PcgState *st) {
  const int c = blockIdx.y;
  if (st && st[c].done) return;
  for (int64_t i = offI + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    z[c * ldz + i] += w1 * sres[c * n + i] * dinv[i - offI];
}

// coarse correction d = R_W^T zW (d zero elsewhere beforehand), z += d
__global__ void k_coarse_scatter2_m(int nW, int npad, const int32_t *__restrict__ wd, const double *__restrict__ zW,
                                    int64_t n, double *__restrict__ d, double *__restrict__ z, int64_t ldz,
                                    const PcgState *st, double wscale) {
  const int c = blockIdx.y;
  if (st && st[c].done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nW) {
    const double v = wscale * zW[int64_t(c) * npad + i];
    d[c * n + wd[i]] = v;
    z[c * ldz + wd[i]] += v;
  }
}

// y = a x + b y on one vector (setup-time Krylov steps)
__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b, double *__restrict__ y) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

// zero y outside [lo, hi)
__global__ void k_mask(int64_t n, int64_t lo, int64_t hi, double *__restrict__ y) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    if (i < lo || i >= hi) y[i] = 0.0;
}

}  // namespace

// ================================================================ launchers
void launch_weights(int d, int k, int64_t n_cells, const double *X, const double *Einv, double alpha, double beta,
                    double *w, int Q, hipStream_t s) {
  hipLaunchKernelGGL(k_weights, dim3(grid_for(n_cells, 128)), dim3(128), 0, s, d, k, n_cells, X, Einv, alpha, beta,
                     w, Q);
}

void launch_interior_diag(int64_t n_cells, int n, int Q, const double *R, const double *w, const int32_t *cell_dofs,
                          const int32_t *loc_interior, int n_int_loc, int64_t off_I, double *dinv, hipStream_t s) {
  if (n_int_loc == 0) return;
  hipLaunchKernelGGL(k_interior_diag, dim3(grid_for(n_cells * n_int_loc, 256)), dim3(256), 0, s, n_cells, n, Q, R,
                     w, cell_dofs, loc_interior, n_int_loc, off_I, dinv);
}

void launch_pad_identity(int64_t B, int N, const int32_t *sizes, double *A, hipStream_t s) {
  hipLaunchKernelGGL(k_pad_identity, dim3(unsigned(B)), dim3(64), 0, s, B, N, sizes, A);
}

void launch_patch_assemble(int64_t n_items, const int32_t *item_patch, const int32_t *item_cell,
                           const int64_t *item_trip, const int32_t *tr_col, const int32_t *tr_loc,
                           const double *tr_coef, int n, int Q, const double *R, const double *w, int N, double *A,
                           hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_patch_assemble, dim3(unsigned(n_items)), dim3(256), 0, s, item_patch, item_cell, item_trip,
                     tr_col, tr_loc, tr_coef, n, Q, R, w, N, A);
}

// blocks a trtri step aims for before its sums are split
constexpr int64_t kTrtriBlocks = 4096;

int64_t chol_inverse_work(int64_t B, int N) {
  const int NB = N / BS;
  int64_t most = 0;
  for (int st = 1; st < NB; ++st) {
    const int64_t tiles = int64_t(NB - st) * B;
    if (tiles >= kTrtriBlocks) continue;
    const int nK = int(std::min<int64_t>(st, (kTrtriBlocks + tiles - 1) / tiles));
    if (nK > 1) most = std::max(most, tiles * nK);
  }
  return most * BS * BS;
}

void launch_chol_inverse(int64_t B, int N, double *A, double *Linv, int *status, double *work, hipStream_t s) {
  const int NB = N / BS;
  for (int kb = 0; kb < NB; ++kb) {
    hipLaunchKernelGGL(k_chol_diag, dim3(unsigned(B)), dim3(256), 0, s, N, kb, A, status);
    const int m = NB - kb - 1;
    if (m > 0) {
      hipLaunchKernelGGL(k_chol_panel, dim3(m, unsigned(B)), dim3(256), 0, s, N, kb, A);
      hipLaunchKernelGGL(k_chol_update, dim3(unsigned(int64_t(m) * (m + 1) / 2), unsigned(B)), dim3(256), 0, s, N,
                         kb, A);
    }
  }
  hipLaunchKernelGGL(k_trtri_diag, dim3(unsigned(NB), unsigned(B)), dim3(256), 0, s, N, A, Linv);
  for (int st = 1; st < NB; ++st) {
    const int64_t tiles = int64_t(NB - st) * B;
    int nK = tiles >= kTrtriBlocks ? 1 : int(std::min<int64_t>(st, (kTrtriBlocks + tiles - 1) / tiles));
    if (nK > 1 && work) {
      const int KC = (st + nK - 1) / nK;
      nK = (st + KC - 1) / KC;
      hipLaunchKernelGGL(k_trtri_part, dim3(unsigned(NB - st), unsigned(nK), unsigned(B)), dim3(256), 0, s, N, st,
                         KC, nK, A, Linv, work);
      hipLaunchKernelGGL(k_trtri_fin, dim3(unsigned(NB - st), unsigned(B)), dim3(256), 0, s, N, st, nK, work, Linv);
    } else {
      hipLaunchKernelGGL(k_trtri_step, dim3(unsigned(NB - st), unsigned(B)), dim3(256), 0, s, N, st, A, Linv);
    }
  }
  hipLaunchKernelGGL(k_lauum, dim3(unsigned(int64_t(NB) * (NB + 1) / 2), unsigned(B)), dim3(256), 0, s, N, Linv, A);
}

void launch_pack_seg(int64_t B, int N, int E, const int32_t *sizes, const int64_t *off, const double *Ainv,
                     double *packed, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_seg, dim3(unsigned(B)), dim3(256), 0, s, N, E, sizes, off, Ainv, packed);
}

void launch_pack_tiles(int N, int n, const double *Ainv, double *tiles, hipStream_t s) {
  const int NT = (n + 63) / 64;
  hipLaunchKernelGGL(k_pack_tiles, dim3(unsigned(int64_t(NT) * (NT + 1) / 2)), dim3(256), 0, s, N, n, NT, Ainv,
                     tiles);
}

template <typename T, int Q>
static void apply_A_q(const ApplyATables &t, int NB, dim3 grid, int kb0, int kb1, const double *x, int64_t ldx,
                      double *y, int64_t ldy, double alpha, const PcgState *st, hipStream_t s, int mb0, int64_t d0,
                      bool overwrite, double *xclr) {
  const int64_t d1 = t.n_dofs;
  const int KB = t.KP / 4;
  const bool full = kb0 == 0 && kb1 == KB && mb0 == 0;
  const int ncol = int(grid.z);
  // FP32: the tables' FP32 copies, and the cell vectors in the first half of
  // the FP64 work buffers
  const T *Af = sizeof(T) == 8 ? (const T *)t.Afrag : (const T *)t.Afrag32;
  const T *w = sizeof(T) == 8 ? (const T *)t.w : (const T *)t.w32;
  T *Xc = reinterpret_cast<T *>(t.Xc), *Yc = reinterpret_cast<T *>(t.Yc);
  hipLaunchKernelGGL(k_gather_cells<T>, dim3(grid_for(int64_t(kb1 - kb0) * t.ncp * 4, 256, 4096), ncol), dim3(256),
                     0, s, t.n, t.KP, t.n_cells, t.ncp, kb0, kb1, t.cell_dofs, x, ldx, Xc, st, t.dmask);
#define RZ_A64(NBV, F)                                                                                        \
  hipLaunchKernelGGL((k_apply_A<T, Q, NBV, F>), grid, dim3(256), 0, s, mb0, KB, kb0, kb1, t.n_cells, t.ncp,  \
                     Af, w, Xc, Yc, t.KP, t.NP, st)
  if (full) {
    if (NB == 4) RZ_A64(4, true);
    else if (NB == 2) RZ_A64(2, true);
    else RZ_A64(1, true);
  } else {
    if (NB == 4) RZ_A64(4, false);
    else if (NB == 2) RZ_A64(2, false);
    else RZ_A64(1, false);
  }
#undef RZ_A64
  if (d1 > d0)
    hipLaunchKernelGGL(k_assemble<T>, dim3(grid_for(d1 - d0, 256, 4096), ncol), dim3(256), 0, s, d0, d1, t.asm_ptr,
                       t.asm_ent, int64_t(t.NP) * t.ncp, Yc, y, ldy, alpha, overwrite ? 1 : 0, xclr, ldx, st,
                       t.dmask);
}

void launch_apply_A(const ApplyATables &t, const double *x, int64_t ldx, double *y, int64_t ldy, int n_rhs,
                    const PcgState *st, hipStream_t s, bool lo, int col0, int col1, double alpha, int row0,
                    int64_t dof0, bool overwrite, bool clear_x) {
  if (col1 < 0) col1 = t.n;
  if (col0 >= col1) {
    if (overwrite) launch_fill(y, t.n_dofs, ldy, n_rhs, st, s);
    if (clear_x) launch_fill(const_cast<double *>(x), t.n_dofs, ldx, n_rhs, st, s);
    return;
  }
  const int kb0 = col0 / 4, kb1 = (col1 + 3) / 4;
  const int NMB = t.NP / 16;
  const int mb0 = row0 / 16;
  // cells per wave: as many as keep >= 2048 waves in flight (A-fragment reuse
  // vs occupancy), counting the row blocks this launch covers; an apply over
  // all rows of one column takes the tuned value where there is one
  int NB = 4;
  while (NB > 1 && ((t.n_cells + 16 * NB - 1) / (16 * NB)) * (NMB - mb0) * n_rhs < 2048) NB /= 2;
  if (n_rhs == 1 && mb0 == 0 && (t.nb1 == 1 || t.nb1 == 2 || t.nb1 == 4)) NB = t.nb1;
  if (t.nb_all == 1 || t.nb_all == 2 || t.nb_all == 4) NB = t.nb_all;
  // GEMM: a block is one row block x 4 waves x 16 NB cells; a row-
  // restricted apply starts at the row block of row0 and assembles the dofs
  // from dof0 on (the interior rows and dofs: both are trailing blocks)
  const dim3 g64(unsigned((t.n_cells + 64 * NB - 1) / (64 * NB)), unsigned(NMB - mb0), unsigned(n_rhs));
  double *xclr = clear_x ? const_cast<double *>(x) : nullptr;
#define RZ_AQ(TT)                                                                                               \
  do {                                                                                                          \
    if (t.Q == 12) apply_A_q<TT, 12>(t, NB, g64, kb0, kb1, x, ldx, y, ldy, alpha, st, s, mb0, dof0, overwrite, xclr); \
    else if (t.Q == 7) apply_A_q<TT, 7>(t, NB, g64, kb0, kb1, x, ldx, y, ldy, alpha, st, s, mb0, dof0, overwrite, xclr); \
    else apply_A_q<TT, 4>(t, NB, g64, kb0, kb1, x, ldx, y, ldy, alpha, st, s, mb0, dof0, overwrite, xclr);      \
  } while (0)
  if (lo && t.Afrag32) RZ_AQ(float);
  else RZ_AQ(double);
#undef RZ_AQ
}

// patch apply: largest G in {8,4,2,1} with G <= ncol, LDS <= 96 KB, MAXJ * G <= 32
int64_t seg_size(int m, int V) {
  const int64_t mS = (m + V - 1) / V * V;
  return seg_row_off(m, mS, V);
}

int64_t fold_size(int m, int esize) { return int64_t((m + 1) / 2 + 1) * 2 * fold_hp(m, esize); }

void launch_pack_fold(int64_t B, int N, const int32_t *sizes, const int64_t *off, const double *Ainv,
                      double *packed, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_fold, dim3(unsigned(B)), dim3(256), 0, s, N, sizes, off, Ainv, packed);
}

void launch_seg_to_float(int64_t n_patches, const int64_t *patch_col, const int64_t *off64, const int64_t *off32,
                         const double *A, float *B, bool fold, hipStream_t s) {
  if (fold)
    hipLaunchKernelGGL((k_fold_to_low<float, 4>), dim3(unsigned(n_patches)), dim3(256), 0, s, patch_col, off64,
                       off32, A, B);
  else
    hipLaunchKernelGGL((k_seg_to_low<float, 4>), dim3(unsigned(n_patches)), dim3(256), 0, s, patch_col, off64,
                       off32, A, B);
}
void launch_seg_to_bf16(int64_t n_patches, const int64_t *patch_col, const int64_t *off64, const int64_t *off16,
                        const double *A, uint16_t *B, bool fold, hipStream_t s) {
  if (fold)
    hipLaunchKernelGGL((k_fold_to_low<uint16_t, 8>), dim3(unsigned(n_patches)), dim3(256), 0, s, patch_col, off64,
                       off16, A, B);
  else
    hipLaunchKernelGGL((k_seg_to_low<uint16_t, 8>), dim3(unsigned(n_patches)), dim3(256), 0, s, patch_col, off64,
                       off16, A, B);
}

// rows in flight per lane group: deeper for short rows
template <int VQ, typename T>
constexpr int patch_depth() {
  // FP64 and FP32 variants with 16 or more values per lane per row (patches
  // of 513-2048 dofs) keep no row in flight ahead: their two row buffers cost
  // occupancy.  FP64 with 16 stripes took 256 VGPRs and spilled to AGPRs (one
  // wave per SIMD; with one buffer 228 VGPRs, two waves, applies 24-37%
  // faster); FP64 with 8 stripes 160 VGPRs (three waves; with one buffer 119,
  // four waves, 1.5-2.5% faster); FP32 applies got 23-35% (1025-2048 dofs)
  // and 1.5-3% (513-1024 dofs) faster.  bfloat16 rows are a quarter of the
  // bytes and keep their two buffers: with one the widest variant ran 11%
  // slower.
  return VQ <= 8 ? 4 : (sizeof(T) >= 4 ? 1 : 2);
}

template <int V, int L, int NQ, int G, typename T, int NW, bool NT>
static void patch_seg_nt(const PatchApply &pa, const int64_t *off, const T *inv, dim3 grid, size_t lds,
                         const double *r, int64_t ldr, double *z, int64_t ldz, int ncol, double scale,
                         const PcgState *st, hipStream_t s) {
  constexpr int D = patch_depth<NQ * V, T>();
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void *)k_patch_seg<V, L, NQ, G, D, T, NW, NT>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  hipLaunchKernelGGL((k_patch_seg<V, L, NQ, G, D, T, NW, NT>), grid, dim3(64 * NW), lds, s, pa.chunk_patch,
                     pa.chunk_rows, pa.patch_col, pa.col_ent, pa.ent_dof, pa.ent_coef, off, inv, r, ldr, z, ldz,
                     ncol, scale, st);
}


template <int V, int L, int NQ, int G, typename T, int NW>
static void patch_seg_g(const PatchApply &pa, const int64_t *off, const T *inv, dim3 grid, size_t lds,
                        const double *r, int64_t ldr, double *z, int64_t ldz, int ncol, double scale,
                        const PcgState *st, hipStream_t s) {
  if (pa.n_entries * int64_t(sizeof(T)) > kStreamBytes)
    patch_seg_nt<V, L, NQ, G, T, NW, true>(pa, off, inv, grid, lds, r, ldr, z, ldz, ncol, scale, st, s);
  else
    patch_seg_nt<V, L, NQ, G, T, NW, false>(pa, off, inv, grid, lds, r, ldr, z, ldz, ncol, scale, st, s);
}

template <int V, int L, int NQ, typename T, int NW>
static void patch_seg_w(const PatchApply &pa, const int64_t *off, const T *inv, const double *r, int64_t ldr,
                        double *z, int64_t ldz, int ncol, double scale, const PcgState *st, hipStream_t s) {
  constexpr int W = NQ * L * V;
  constexpr int VQ = NQ * V;
  const size_t lds_per_g = size_t(1 + NW) * W * sizeof(double);
  int G = 4;
  while (G > 1 && (G > ncol || lds_per_g * G > 96 * 1024 || VQ * G > 32)) G /= 2;
  const dim3 grid(unsigned(pa.n_chunks), unsigned((ncol + G - 1) / G));
  if (G == 4)
    patch_seg_g<V, L, NQ, (VQ <= 8 ? 4 : 1), T, NW>(pa, off, inv, grid, lds_per_g * G, r, ldr, z, ldz, ncol, scale,
                                                    st, s);
  else if (G == 2)
    patch_seg_g<V, L, NQ, (VQ <= 16 ? 2 : 1), T, NW>(pa, off, inv, grid, lds_per_g * G, r, ldr, z, ldz, ncol,
                                                     scale, st, s);
  else patch_seg_g<V, L, NQ, 1, T, NW>(pa, off, inv, grid, lds_per_g, r, ldr, z, ldz, ncol, scale, st, s);
}

// bfloat16 patches of up to 128 columns: one wave per block (four times the
// independent patches in flight per CU, hiding the latency of the gather and
// scatter chains that dominate such short streams); else four waves
template <int V, int L, int NQ, typename T>
static void patch_seg(const PatchApply &pa, const int64_t *off, const T *inv, const double *r, int64_t ldr,
                      double *z, int64_t ldz, int ncol, double scale, const PcgState *st, hipStream_t s) {
  if constexpr (sizeof(T) == 2 && L == 16)
    return patch_seg_w<V, L, NQ, T, 1>(pa, off, inv, r, ldr, z, ldz, ncol, scale, st, s);
  else
    patch_seg_w<V, L, NQ, T, 4>(pa, off, inv, r, ldr, z, ldz, ncol, scale, st, s);
}

// lanes per row and column stripes for the largest patch of a set
template <typename T>
static void patch_dispatch(const PatchApply &pa, const int64_t *off, const T *inv, const double *r, int64_t ldr,
                           double *z, int64_t ldz, int ncol, double scale, const PcgState *st, hipStream_t s) {
  constexpr int V = 16 / sizeof(T);
  // kMaxPatch = 2048 columns need at most NQ = 2048 / (64 V) stripes
  static_assert(kMaxPatch <= 64 * 32, "patch stripes cover at most 64 * 32 columns");
  const int m = pa.max_size;
  // 16 lanes per row up to 48 / 64 / 128 columns (V = 2 / 4 / 8), 32 up to
  // 256, else 64 (measured over the patch sets of the 3D sweep problems)
  constexpr int m16 = V == 2 ? 48 : V == 4 ? 64 : 128;
  const int L = m <= m16 ? 16 : (m <= 256 ? 32 : 64);
  const int mS = (m + V - 1) / V * V;
  const int nq = (mS + V * L - 1) / (V * L);
  const int NQ = nq <= 1 ? 1 : nq <= 2 ? 2 : nq <= 4 ? 4 : nq <= 8 ? 8 : 16;
#define RZ_PQ(LL, QQ)                                                                          \
  if constexpr (QQ * V <= 32)                                                                  \
    if (L == LL && NQ == QQ) return patch_seg<V, LL, QQ, T>(pa, off, inv, r, ldr, z, ldz, ncol, scale, st, s)
  RZ_PQ(16, 1); RZ_PQ(16, 2); RZ_PQ(16, 4);
  RZ_PQ(32, 1); RZ_PQ(32, 2); RZ_PQ(32, 4);
  RZ_PQ(64, 1); RZ_PQ(64, 2); RZ_PQ(64, 4); RZ_PQ(64, 8); RZ_PQ(64, 16);
#undef RZ_PQ
  // 64 lanes with 32 / V stripes cover any patch up to kMaxPatch
  patch_seg<V, 64, 32 / V, T>(pa, off, inv, r, ldr, z, ldz, ncol, scale, st, s);
}

template <int V, int L, int NQ, int G, typename T, bool NT>
static void patch_fold_nt(const PatchApply &pa, const int64_t *off, const T *inv, dim3 grid, size_t lds,
                          const double *r, int64_t ldr, double *z, int64_t ldz, int ncol, double scale,
                          const PcgState *st, hipStream_t s) {
#ifdef RZ_FOLD_D
  constexpr int D = RZ_FOLD_D;
#else
  constexpr int D = patch_depth<2 * NQ * V, T>();
#endif
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void *)k_patch_fold<V, L, NQ, G, D, T, 4, NT>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  hipLaunchKernelGGL((k_patch_fold<V, L, NQ, G, D, T, 4, NT>), grid, dim3(256), lds, s, pa.chunk_patch,
                     pa.chunk_rows, pa.patch_col, pa.col_ent, pa.ent_dof, pa.ent_coef, off, inv, r, ldr, z, ldz,
                     ncol, scale, st);
}

template <int V, int L, int NQ, int G, typename T>
static void patch_fold_g(const PatchApply &pa, const int64_t *off, const T *inv, dim3 grid, size_t lds,
                         const double *r, int64_t ldr, double *z, int64_t ldz, int ncol, double scale,
                         const PcgState *st, hipStream_t s) {
  if (pa.n_entries * int64_t(sizeof(T)) > kStreamBytes)
    patch_fold_nt<V, L, NQ, G, T, true>(pa, off, inv, grid, lds, r, ldr, z, ldz, ncol, scale, st, s);
  else
    patch_fold_nt<V, L, NQ, G, T, false>(pa, off, inv, grid, lds, r, ldr, z, ldz, ncol, scale, st, s);
}

// right-hand sides per block as for the segmented kernel, counting the four
// per-position register arrays (2 NQ V values per array pair)
template <int V, int L, int NQ, typename T>
static void patch_fold_w(const PatchApply &pa, const int64_t *off, const T *inv, const double *r, int64_t ldr,
                         double *z, int64_t ldz, int ncol, double scale, const PcgState *st, hipStream_t s) {
  constexpr int W2 = 2 * NQ * L * V;
  constexpr int VQ2 = 2 * NQ * V;
  const size_t lds_per_g = size_t(1 + 4) * W2 * sizeof(double);
  int G = 4;
  while (G > 1 && (G > ncol || lds_per_g * G > 96 * 1024 || VQ2 * G > 32)) G /= 2;
  const dim3 grid(unsigned(pa.n_chunks), unsigned((ncol + G - 1) / G));
  if (G == 4)
    patch_fold_g<V, L, NQ, (VQ2 <= 8 ? 4 : 1), T>(pa, off, inv, grid, lds_per_g * G, r, ldr, z, ldz, ncol, scale,
                                                   st, s);
  else if (G == 2)
    patch_fold_g<V, L, NQ, (VQ2 <= 16 ? 2 : 1), T>(pa, off, inv, grid, lds_per_g * G, r, ldr, z, ldz, ncol,
                                                    scale, st, s);
  else patch_fold_g<V, L, NQ, 1, T>(pa, off, inv, grid, lds_per_g, r, ldr, z, ldz, ncol, scale, st, s);
}

// lanes per pair row and stripes covering hP positions of the largest patch
template <typename T>
static void fold_dispatch(const PatchApply &pa, const int64_t *off, const T *inv, const double *r, int64_t ldr,
                          double *z, int64_t ldz, int ncol, double scale, const PcgState *st, hipStream_t s) {
  constexpr int V = 16 / sizeof(T);
  static_assert(kMaxPatch / 2 <= 64 * 16, "fold stripes cover at most 64 * 16 V positions");
  const int hP = fold_hp(pa.max_size, int(sizeof(T)));
  const int L = hP <= 16 * V ? 16 : (hP <= 32 * V ? 32 : 64);
  const int nq = (hP + V * L - 1) / (V * L);
  const int NQ = nq <= 1 ? 1 : nq <= 2 ? 2 : nq <= 4 ? 4 : nq <= 8 ? 8 : 16;
#define RZ_FQ(LL, QQ)                                                                          \
  if constexpr (QQ * V <= 16)                                                                  \
    if (L == LL && NQ == QQ) return patch_fold_w<V, LL, QQ, T>(pa, off, inv, r, ldr, z, ldz, ncol, scale, st, s)
  RZ_FQ(16, 1); RZ_FQ(32, 1); RZ_FQ(64, 1); RZ_FQ(64, 2); RZ_FQ(64, 4); RZ_FQ(64, 8);
#undef RZ_FQ
  patch_fold_w<V, 64, 16 / V, T>(pa, off, inv, r, ldr, z, ldz, ncol, scale, st, s);
}

template <typename T>
static void patch_any(const PatchApply &pa, const int64_t *off, const T *inv, const double *r, int64_t ldr,
                      double *z, int64_t ldz, int ncol, double scale, const PcgState *st, hipStream_t s) {
  if (pa.fold) fold_dispatch<T>(pa, off, inv, r, ldr, z, ldz, ncol, scale, st, s);
  else patch_dispatch<T>(pa, off, inv, r, ldr, z, ldz, ncol, scale, st, s);
}

template <typename F>
static void patch_mfma(const PatchApply &pa, const F *frag, const int64_t *frag_off, const double *r, int64_t ldr,
                       int ncol, const PcgState *st, hipStream_t s) {
  typedef typename FragTraits<F>::Z_t Z_t;
  constexpr int MPA = FragTraits<F>::MPA;
  const int MP = (pa.max_size + MPA - 1) / MPA * MPA;
  const size_t lds = size_t(MP) * 68 * (sizeof(F) == 8 ? 8 : 4);  // FP64 units, FP32 units, 8-half units / 2
  hipLaunchKernelGGL(k_patch_rt, dim3(unsigned((pa.n_adof + 63) / 64), unsigned((ncol + 63) / 64)), dim3(256), 0,
                     s, pa.n_adof, pa.adof, r, ldr, ncol, static_cast<double *>(pa.rt), pa.zb_cols);
  const dim3 grid(unsigned(pa.n_patches), unsigned((ncol + 63) / 64));
  Z_t *zb = static_cast<Z_t *>(pa.zb);
#define RZ_PM(MM)                                                                                               \
  if (MP <= MM) {                                                                                               \
    static bool attr = false;                                                                                   \
    if (!attr) {                                                                                                \
      (void)hipFuncSetAttribute((const void *)k_patch_mfma<F, MM>, hipFuncAttributeMaxDynamicSharedMemorySize,  \
                                160 * 1024);                                                                    \
      attr = true;                                                                                              \
    }                                                                                                           \
    hipLaunchKernelGGL((k_patch_mfma<F, MM>), grid, dim3(64 * (MM / 16)), lds, s, pa.patch_col, pa.col_ent,     \
                       pa.ent_a, pa.ent_coef, frag_off, frag, static_cast<const double *>(pa.rt), zb, pa.zb_cols, \
                       ncol, st);                                                                               \
    return;                                                                                                     \
  }
  RZ_PM(32) RZ_PM(64) RZ_PM(96) RZ_PM(128)
#undef RZ_PM
}

template <typename Z>
static void patch_zb_scatter(const PatchApply &pa, double *z, int64_t ldz, int ncol, double scale,
                             const PcgState *st, hipStream_t s) {
  hipLaunchKernelGGL((k_patch_zb_scatter<Z>), dim3(unsigned((pa.n_adof + 63) / 64), unsigned((ncol + 63) / 64)),
                     dim3(256), 0, s, pa.n_adof, pa.adof, pa.aptr, pa.apr, pa.acoef, static_cast<const Z *>(pa.zb),
                     pa.zb_cols, z, ldz, ncol, scale, st);
}

void launch_seg_to_frag(const PatchApply &pa, int kind, void *frag, const int64_t *frag_off, hipStream_t s) {
  if (kind == 1)
    hipLaunchKernelGGL((k_seg_to_frag<uint16_t>), dim3(unsigned(pa.n_patches)), dim3(256), 0, s, pa.patch_col,
                       pa.inv_off, pa.inv, frag_off, static_cast<uint16_t *>(frag));
  else if (kind == 2)
    hipLaunchKernelGGL((k_seg_to_frag<float>), dim3(unsigned(pa.n_patches)), dim3(256), 0, s, pa.patch_col,
                       pa.inv_off, pa.inv, frag_off, static_cast<float *>(frag));
  else
    hipLaunchKernelGGL((k_seg_to_frag<double>), dim3(unsigned(pa.n_patches)), dim3(256), 0, s, pa.patch_col,
                       pa.inv_off, pa.inv, frag_off, static_cast<double *>(frag));
}

int64_t frag_size(int m, int kind) {
  const int64_t a = kind == 1 ? 32 : 16, MP = (m + a - 1) / a * a;
  return MP * MP;
}

void launch_patch_apply(const PatchApply &pa, const double *r, int64_t ldr, double *z, int64_t ldz, int ncol,
                        const PcgState *st, hipStream_t s, bool lo, double scale) {
  if (pa.n_chunks == 0) return;
  if (lo && pa.inv16 && ncol >= 8 && pa.frag16 && pa.zb && ncol <= pa.zb_cols) {
    patch_mfma<uint16_t>(pa, pa.frag16, pa.frag_off16, r, ldr, ncol, st, s);
    return patch_zb_scatter<float>(pa, z, ldz, ncol, scale, st, s);
  }
  if (lo && pa.inv16)
    return patch_any<uint16_t>(pa, pa.inv_off16, pa.inv16, r, ldr, z, ldz, ncol, scale, st, s);
  if (lo && pa.inv32 && ncol >= 8 && pa.frag32 && pa.zb && ncol <= pa.zb_cols) {
    patch_mfma<float>(pa, pa.frag32, pa.frag_off32, r, ldr, ncol, st, s);
    return patch_zb_scatter<float>(pa, z, ldz, ncol, scale, st, s);
  }
  if (lo && pa.inv32)
    return patch_any<float>(pa, pa.inv_off32, pa.inv32, r, ldr, z, ldz, ncol, scale, st, s);
  if (ncol >= 8 && pa.frag64 && pa.zb && ncol <= pa.zb_cols) {
    patch_mfma<double>(pa, pa.frag64, pa.frag_off64, r, ldr, ncol, st, s);
    return patch_zb_scatter<double>(pa, z, ldz, ncol, scale, st, s);
  }
  patch_any<double>(pa, pa.inv_off, pa.inv, r, ldr, z, ldz, ncol, scale, st, s);
}

// ---- Hodge Laplacians: the exterior derivative as CSR, weight scaling,
// MINRES vector kernels
// y = alpha A x (+ y when accumulate), A in CSR: L lanes per row, lane j
// summing entries j, j + L, ... of the row, then a butterfly over the L
// lanes (a fixed order for a given L)
template <int L>
__global__ __launch_bounds__(256) void k_csr_spmv(int64_t n, const int64_t *__restrict__ ptr,
                                                  const int32_t *__restrict__ col, const double *__restrict__ val,
                                                  const double *__restrict__ x, double *__restrict__ y, double alpha,
                                                  int accumulate) {
  const int sub = int(threadIdx.x) & (L - 1);
  const int64_t step = int64_t(gridDim.x) * (blockDim.x / L);
  for (int64_t i = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / L; i < n; i += step) {
    double v = 0.0;
    for (int64_t e = ptr[i] + sub; e < ptr[i + 1]; e += L) v += val[e] * x[col[e]];
#pragma unroll
    for (int o = L / 2; o > 0; o /= 2) v += __shfl_xor(v, o, L);
    if (sub == 0) y[i] = accumulate ? y[i] + alpha * v : alpha * v;
  }
}

// out[c, q] = w[c, q] * (q < qm ? smass : sderiv): the mass family of the
// stacked matrices comes first
__global__ void k_scale_weights(int64_t nc, int Q, int qm, const double *__restrict__ w, double smass, double sderiv,
                                double *__restrict__ out) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nc * Q; i += int64_t(gridDim.x) * blockDim.x)
    out[i] = w[i] * (int(i % Q) < qm ? smass : sderiv);
}

// out = a x + b y + c z (null vectors count as zero; out may alias x)
__global__ void k_lincomb3(int64_t n, double a, const double *x, double b, const double *y, double c,
                           const double *z, double *out) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    double v = 0.0;
    if (x) v += a * x[i];
    if (y) v += b * y[i];
    if (z) v += c * z[i];
    out[i] = v;
  }
}

// out = d .* x (out may alias x)
__global__ void k_diag_mul(int64_t n, const double *d, const double *x, double *out) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    out[i] = d[i] * x[i];
}

// per-block partial sums of a . b (blockDim 256; gridDim.x partials)
__global__ __launch_bounds__(256) void k_dot_part(int64_t n, const double *__restrict__ a,
                                                  const double *__restrict__ b, double *__restrict__ part) {
  __shared__ double sm4[4];
  double v = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) v += a[i] * b[i];
  v = block_sum256(v, sm4);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

void launch_csr_spmv(int64_t n, const int64_t *ptr, const int32_t *col, const double *val, const double *x,
                     double *y, double alpha, bool accumulate, int lanes, hipStream_t s) {
  if (n <= 0) return;
  const int L = lanes >= 64 ? 64 : lanes >= 16 ? 16 : lanes >= 4 ? 4 : 1;
  const unsigned g = unsigned(std::min<int64_t>((n * L + 255) / 256, 8192));
  const int acc = accumulate ? 1 : 0;
  if (L == 64) hipLaunchKernelGGL(k_csr_spmv<64>, dim3(g), dim3(256), 0, s, n, ptr, col, val, x, y, alpha, acc);
  else if (L == 16) hipLaunchKernelGGL(k_csr_spmv<16>, dim3(g), dim3(256), 0, s, n, ptr, col, val, x, y, alpha, acc);
  else if (L == 4) hipLaunchKernelGGL(k_csr_spmv<4>, dim3(g), dim3(256), 0, s, n, ptr, col, val, x, y, alpha, acc);
  else hipLaunchKernelGGL(k_csr_spmv<1>, dim3(g), dim3(256), 0, s, n, ptr, col, val, x, y, alpha, acc);
}
void launch_scale_weights(int64_t nc, int Q, int qm, const double *w, double smass, double sderiv, double *out,
                          hipStream_t s) {
  const unsigned g = unsigned(std::min<int64_t>((nc * Q + 255) / 256, 8192));
  hipLaunchKernelGGL(k_scale_weights, dim3(g), dim3(256), 0, s, nc, Q, qm, w, smass, sderiv, out);
}
void launch_lincomb3(int64_t n, double a, const double *x, double b, const double *y, double c, const double *z,
                     double *out, hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = unsigned(std::min<int64_t>((n + 255) / 256, 8192));
  hipLaunchKernelGGL(k_lincomb3, dim3(g), dim3(256), 0, s, n, a, x, b, y, c, z, out);
}
void launch_diag_mul(int64_t n, const double *d, const double *x, double *out, hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = unsigned(std::min<int64_t>((n + 255) / 256, 8192));
  hipLaunchKernelGGL(k_diag_mul, dim3(g), dim3(256), 0, s, n, d, x, out);
}
void launch_dot_part(int64_t n, const double *a, const double *b, double *part, int nparts, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_part, dim3(unsigned(nparts)), dim3(256), 0, s, n, a, b, part);
}

// ---- geometric multigrid V-cycle on W^k (small sparse levels; one thread
// per row, columns in blockIdx.y)
// t = b - A x (and z = 0 when zero_z: the edge-star relaxation accumulates there)
__global__ void k_mg_resid(int64_t n, const int64_t *__restrict__ ap, const int32_t *__restrict__ ac,
                           const double *__restrict__ av, const double *__restrict__ b, int64_t ldb,
                           const double *__restrict__ x, int64_t ldx, double *__restrict__ t, double *__restrict__ z) {
  const int c = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double *xc = x + c * ldx;
  double sum = 0.0;
  for (int64_t e = ap[i]; e < ap[i + 1]; ++e) sum += av[e] * xc[ac[e]];
  t[c * n + i] = b[c * ldb + i] - sum;
  if (z) z[c * n + i] = 0.0;
}
// y = A x (add: y += A x), y with leading dimension ldy
__global__ void k_mg_spmv(int64_t n, int64_t nx, const int64_t *__restrict__ ap, const int32_t *__restrict__ ac,
                          const double *__restrict__ av, const double *__restrict__ x, double *__restrict__ y,
                          int64_t ldy, int add) {
  const int c = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double *xc = x + c * nx;
  double sum = 0.0;
  for (int64_t e = ap[i]; e < ap[i + 1]; ++e) sum += av[e] * xc[ac[e]];
  y[c * ldy + i] = add ? y[c * ldy + i] + sum : sum;
}
// point-Jacobi step x += omega dinv t
__global__ void k_mg_jacobi(int64_t n, const double *__restrict__ dinv, double omega, const double *__restrict__ t,
                            double *__restrict__ x, int64_t ldx) {
  const int c = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[c * ldx + i] += omega * dinv[i] * t[c * n + i];
}
// Hiptmair-Jacobi, vertex part: u_v = gdiag_v (G^T t)_v
__global__ void k_mg_grad_t(int64_t nv, int64_t n, const int64_t *__restrict__ gp, const int32_t *__restrict__ gc,
                            const double *__restrict__ gv, const double *__restrict__ gdiag,
                            const double *__restrict__ t, double *__restrict__ u) {
  const int c = blockIdx.y;
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double sum = 0.0;
  for (int64_t e = gp[v]; e < gp[v + 1]; ++e) sum += gv[e] * t[c * n + gc[e]];
  u[c * nv + v] = gdiag[v] * sum;
}
// Hiptmair-Jacobi step: x += omega (dinv t + G u)
__global__ void k_mg_hiptmair(int64_t n, int64_t nv, const double *__restrict__ dinv, const int64_t *__restrict__ gp,
                              const int32_t *__restrict__ gc, const double *__restrict__ gv, double omega,
                              const double *__restrict__ t, const double *__restrict__ u, double *__restrict__ x,
                              int64_t ldx) {
  const int c = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = dinv[i] * t[c * n + i];
  for (int64_t e = gp[i]; e < gp[i + 1]; ++e) s += gv[e] * u[c * nv + gc[e]];
  x[c * ldx + i] += omega * s;
}
// edge-star relaxation: z[faces of E] += A_E^{-1} t[faces of E], one thread per star
__global__ void k_mg_stars(int64_t nstar, int64_t n, const int64_t *__restrict__ sp, const int32_t *__restrict__ sf,
                           const int64_t *__restrict__ so, const double *__restrict__ sinv, const double *__restrict__ t,
                           double *__restrict__ z) {
  const int c = blockIdx.y;
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nstar) return;
  const int64_t f0 = sp[e];
  const int m = int(sp[e + 1] - f0);
  const double *Ai = sinv + so[e];
  double tl[8];
  for (int a = 0; a < m && a < 8; ++a) tl[a] = t[c * n + sf[f0 + a]];
  for (int a = 0; a < m && a < 8; ++a) {
    double acc = 0.0;
    for (int b = 0; b < m && b < 8; ++b) acc += Ai[a * m + b] * tl[b];
    atomicAdd(&z[c * n + sf[f0 + a]], acc);
  }
}
__global__ void k_mg_axpy(int64_t n, double omega, const double *__restrict__ z, double *__restrict__ x, int64_t ldx) {
  const int c = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[c * ldx + i] += omega * z[c * n + i];
}
// coarsest level: x = cinv b (dense, row-major)
__global__ void k_mg_dense(int64_t n, const double *__restrict__ cinv, const double *__restrict__ b, int64_t ldb,
                           double *__restrict__ x, int64_t ldx) {
  const int c = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t j = 0; j < n; ++j) s += cinv[i * n + j] * b[c * ldb + j];
  x[c * ldx + i] = s;
}

static void mg_level(const MgDev &mg, int l, const double *b, int64_t ldb, double *x, int64_t ldx, int ncol,
                     hipStream_t s) {
  const MgDevLevel &L = mg.lev[l];
  const int64_t n = L.n;
  const dim3 gn(grid_for(n, 256), ncol);
  if (l == mg.L - 1) {
    hipLaunchKernelGGL(k_mg_dense, gn, dim3(256), 0, s, n, mg.cinv, b, ldb, x, ldx);
    return;
  }
  hipLaunchKernelGGL(k_fill_m, dim3(grid_for(n, 256, 2048), ncol), dim3(256), 0, s, x, n, ldx, nullptr);
  auto smooth = [&]() {
    hipLaunchKernelGGL(k_mg_resid, gn, dim3(256), 0, s, n, L.Ap, L.Ac, L.Av, b, ldb, x, ldx, L.t,
                       mg.k == 2 ? L.z : nullptr);
    if (mg.k == 0) {
      hipLaunchKernelGGL(k_mg_jacobi, gn, dim3(256), 0, s, n, L.dinv, L.omega, L.t, x, ldx);
    } else if (mg.k == 1) {
      hipLaunchKernelGGL(k_mg_grad_t, dim3(grid_for(L.nv, 256), ncol), dim3(256), 0, s, L.nv, n, L.Gtp, L.Gtc,
                         L.Gtv, L.gdiag, L.t, L.u);
      hipLaunchKernelGGL(k_mg_hiptmair, gn, dim3(256), 0, s, n, L.nv, L.dinv, L.Gp, L.Gc, L.Gv, L.omega, L.t, L.u, x,
                         ldx);
    } else {
      hipLaunchKernelGGL(k_mg_stars, dim3(grid_for(L.nstar, 128), ncol), dim3(128), 0, s, L.nstar, n, L.sp, L.sf,
                         L.so, L.sinv, L.t, L.z);
      hipLaunchKernelGGL(k_mg_axpy, gn, dim3(256), 0, s, n, L.omega, L.z, x, ldx);
    }
  };
  for (int k = 0; k < mg.nu; ++k) smooth();
  hipLaunchKernelGGL(k_mg_resid, gn, dim3(256), 0, s, n, L.Ap, L.Ac, L.Av, b, ldb, x, ldx, L.t, nullptr);
  const MgDevLevel &C = mg.lev[l + 1];
  hipLaunchKernelGGL(k_mg_spmv, dim3(grid_for(C.n, 256), ncol), dim3(256), 0, s, C.n, n, L.Rp, L.Rc, L.Rv, L.t, C.b,
                     C.n, 0);
  mg_level(mg, l + 1, C.b, C.n, C.x, C.n, ncol, s);
  hipLaunchKernelGGL(k_mg_spmv, gn, dim3(256), 0, s, n, C.n, L.Pp, L.Pc, L.Pv, C.x, x, ldx, 1);
  for (int k = 0; k < mg.nu; ++k) smooth();
}

void launch_mg_cycle(const MgDev &mg, const double *b0, int64_t ldb0, double *x0, int64_t ldx0, int ncol,
                     hipStream_t s) {
  mg_level(mg, 0, b0, ldb0, x0, ldx0, ncol, s);
}

void launch_coarse_tiles(const CoarseApply &ca, int ncol, const PcgState *st, hipStream_t s, bool lo) {
  if (ca.mg) {
    launch_mg_cycle(*ca.mg, ca.rW, int64_t(ca.NT) * 64, ca.zW, int64_t(ca.NT) * 64, ncol, s);
    return;
  }
  const unsigned nt = unsigned(int64_t(ca.NT) * (ca.NT + 1) / 2);
  const int npad = ca.NT * 64;
  if (ncol >= 8 && ca.full) {
    // split the block-row sum so that there are >= ~1024 blocks
    const int cgs = (ncol + 63) / 64;
    int nsplit = std::max(1, std::min(ca.NT, 1024 / std::max(1, ca.NT * cgs)));
    hipLaunchKernelGGL(k_coarse_gemm, dim3(ca.NT, cgs, nsplit), dim3(256), 0, s, ca.NT, nsplit, ca.full, ca.rW,
                       ca.zW, npad, ncol, st);
    return;
  }
  // strips of S tiles per block, >= ~2048 blocks where the matrix allows
  const int S = int(std::max<int64_t>(1, std::min<int64_t>(16, int64_t(nt) / 2048)));
  const int G = ncol >= 2 ? 2 : 1;
  const dim3 g(unsigned(ca.NT), unsigned((ca.NT + S - 1) / S), unsigned((ncol + G - 1) / G));
  const bool f32 = lo && ca.tiles32;
  const bool nts = int64_t(nt) * 4096 * (f32 ? 4 : 8) > kStreamBytes;
#define RZ_CT(GG, TT, TI)                                                                                        \
  do {                                                                                                           \
    if (nts)                                                                                                     \
      hipLaunchKernelGGL((k_coarse_symv<GG, TT, true>), g, dim3(256), 0, s, ca.NT, S, TI, ca.rW, ca.zW, npad, ncol, \
                         st);                                                                                    \
    else                                                                                                         \
      hipLaunchKernelGGL((k_coarse_symv<GG, TT, false>), g, dim3(256), 0, s, ca.NT, S, TI, ca.rW, ca.zW, npad,  \
                         ncol, st);                                                                              \
  } while (0)
  if (f32) {
    if (G == 2) RZ_CT(2, float, ca.tiles32);
    else RZ_CT(1, float, ca.tiles32);
  } else {
    if (G == 2) RZ_CT(2, double, ca.tiles);
    else RZ_CT(1, double, ca.tiles);
  }
#undef RZ_CT
}

void launch_apply_P(const PatchApply *sets, int nsets, const CoarseApply &ca, int64_t n, int64_t off_I,
                    const double *dinv, const double *r, int64_t ldr, double *z, int64_t ldz, int ncol,
                    hipStream_t s, bool lo) {
  hipLaunchKernelGGL(k_jacobi_m, dim3(grid_for(n, 256, 2048), ncol), dim3(256), 0, s, n, off_I, dinv, r, ldr, z, ldz);
  for (int i = 0; i < nsets; ++i) launch_patch_apply(sets[i], r, ldr, z, ldz, ncol, nullptr, s, lo);
  const int npad = ca.NT * 64;
  hipLaunchKernelGGL(k_coarse_gather_m, dim3(grid_for(npad, 256), ncol), dim3(256), 0, s, ca.nW, npad, ca.wdofs, r,
                     ldr, ca.rW, ca.zW, ca.dmask);
  launch_coarse_tiles(ca, ncol, nullptr, s, lo);
  hipLaunchKernelGGL(k_coarse_scatter_m, dim3(grid_for(ca.nW, 256), ncol), dim3(256), 0, s, ca.nW, npad, ca.wdofs,
                     ca.zW, z, ldz);
}

void launch_fill(double *y, int64_t n, int64_t ld, int ncol, const PcgState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_m, dim3(grid_for(n, 256, 2048), ncol), dim3(256), 0, s, y, n, ld, st);
}
void launch_copy(int64_t n, const double *a, int64_t lda, double *b, int64_t ldb, int ncol, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_m, dim3(grid_for(n, 256, 2048), ncol), dim3(256), 0, s, n, a, lda, b, ldb);
}
void launch_residual(int64_t n, const double *b, int64_t ldb, const double *Ax, double *r, int ncol, hipStream_t s) {
  hipLaunchKernelGGL(k_residual_m, dim3(grid_for(n, 256, 2048), ncol), dim3(256), 0, s, n, b, ldb, Ax, r);
}
void launch_dot(int64_t n, const double *a, int64_t lda, const double *b, int64_t ldb, const CoarseFold &cf,
                int npad, double *part, int RB, int ncol, const PcgState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_m, dim3(RB, ncol), dim3(256), 0, s, n, a, lda, b, ldb, cf, npad, part, RB, st);
}
void launch_pcg_start(const double *partB, const double *partR, int RB, double tol2, int maxit, PcgState *st,
                      int ncol, hipStream_t s, const PcgState *outer) {
  hipLaunchKernelGGL(k_pcg_start, dim3(ncol), dim3(256), 0, s, partB, partR, RB, tol2, maxit, st, outer);
}
void launch_update_xr(int64_t n, double *x, int64_t ldx, double *r, const double *p, const double *Ap,
                      const double *partZ, const double *partA, double *partR, int RB, int ncol, PcgState *st,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_update_xr_m, dim3(RB, ncol), dim3(256), 0, s, n, x, ldx, r, p, Ap, partZ, partA, partR, RB,
                     st);
}
void launch_check_jacobi(int64_t n, int64_t off_I, const double *dinv, const double *r, double *z,
                         const CoarseApply &ca, const double *partR, int RB, int ncol, PcgState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_check_jacobi_m, dim3(grid_for(n, 256, std::max(1, 2048 / ncol)), ncol), dim3(256), 0, s, n,
                     off_I, dinv, r, z, ca.nW, ca.NT * 64, ca.wdofs, ca.rW, ca.zW, partR, RB, st);
}
void launch_update_p(int64_t n, double *p, const double *z, const CoarseFold &cf, int npad, double *Ap,
                     const double *partZ, int RB, int ncol, PcgState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_update_p_m, dim3(grid_for(n, 256, std::max(1, 2048 / ncol)), ncol), dim3(256), 0, s, n, p, z,
                     cf, npad, Ap, partZ, RB, st);
}

void launch_coarse_expand(int NT, const double *tiles, double *full, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_expand, dim3(NT, NT), dim3(256), 0, s, NT, tiles, full);
}

void launch_to_float(int64_t n, const double *a, float *b, hipStream_t s) {
  hipLaunchKernelGGL(k_to_float, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, a, b);
}
void launch_axpy(int64_t n, const double *d, double *x, int64_t ldx, int ncol, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_m, dim3(grid_for(n, 256, 2048), ncol), dim3(256), 0, s, n, d, x, ldx);
}

// ---- hybrid sweep
void launch_hyb_init(int64_t n, int64_t off_I, const double *dinv, double w1, const double *r, int64_t ldr, double *z,
                     int64_t ldz, double *sres, double *d, const double *partR, int RB, int ncol, PcgState *st,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_hyb_init_m, dim3(grid_for(n, 256, std::max(1, 2048 / ncol)), ncol), dim3(256), 0, s, n, off_I,
                     dinv, w1, r, ldr, z, ldz, sres, d, partR, RB, st);
}
void launch_add(int64_t n, const double *d, double *z, int64_t ldz, int ncol, const PcgState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_add_m, dim3(grid_for(n, 256, std::max(1, 2048 / ncol)), ncol), dim3(256), 0, s, n, d, z, ldz,
                     st);
}
void launch_jacobi_add(int64_t n, int64_t off_I, const double *dinv, double w1, const double *sres, double *z,
                       int64_t ldz, int ncol, const PcgState *st, hipStream_t s) {
  if (off_I >= n) return;
  hipLaunchKernelGGL(k_jacobi_add_m, dim3(grid_for(n - off_I, 256, std::max(1, 2048 / ncol)), ncol), dim3(256), 0, s,
                     n, off_I, dinv, w1, sres, z, ldz, st);
}
void launch_coarse_gather(const CoarseApply &ca, const double *r, int64_t ldr, int ncol, hipStream_t s) {
  const int npad = ca.NT * 64;
  hipLaunchKernelGGL(k_coarse_gather_m, dim3(grid_for(npad, 256), ncol), dim3(256), 0, s, ca.nW, npad, ca.wdofs, r,
                     ldr, ca.rW, ca.zW, ca.dmask);
}
void launch_coarse_scatter2(const CoarseApply &ca, int64_t n, double *d, double *z, int64_t ldz, int ncol,
                            const PcgState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_scatter2_m, dim3(grid_for(ca.nW, 256), ncol), dim3(256), 0, s, ca.nW, ca.NT * 64,
                     ca.wdofs, ca.zW, n, d, z, ldz, st, ca.wscale);
}
__global__ void k_zero_rows(const int32_t *__restrict__ rows, int64_t nrows, double *__restrict__ y, int64_t ld) {
  const int c = blockIdx.y;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nrows; i += int64_t(gridDim.x) * blockDim.x)
    y[c * ld + rows[i]] = 0.0;
}
void launch_zero_rows(const int32_t *rows, int64_t nrows, double *y, int64_t ld, int ncol, hipStream_t s) {
  if (nrows == 0) return;
  hipLaunchKernelGGL(k_zero_rows, dim3(grid_for(nrows, 256, 1024), ncol), dim3(256), 0, s, rows, nrows, y, ld);
}
__global__ void k_set_diag(int N, const int32_t *__restrict__ idx, int n, double *__restrict__ A) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) A[int64_t(idx[i]) * N + idx[i]] = 1.0;
}
void launch_set_diag(int N, const int32_t *idx, int n, double *A, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_set_diag, dim3(grid_for(n, 256)), dim3(256), 0, s, N, idx, n, A);
}
void launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(n, 256, 2048)), dim3(256), 0, s, n, a, x, b, y);
}
void launch_mask(int64_t n, int64_t lo, int64_t hi, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_mask, dim3(grid_for(n, 256, 2048)), dim3(256), 0, s, n, lo, hi, y);
}

}  // namespace rz
