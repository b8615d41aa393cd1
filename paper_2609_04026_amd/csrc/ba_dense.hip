// Direct solve of the reduced camera / group system: the dense-Schur variant of the
// solver (Sec. 4.1, chosen there for reconstructions with few images).  The damped
// Schur complement S = U + lambda D_A - W V^-1 W^T of Sec. 3.1 Eq. 3 is formed
// explicitly in FP64, factored S = L L^T and solved by two triangular solves.
//
// Assembly.  For a feature f take a factor G_f G_f^T = V_f^-1 of the damped inverse
// that the implicit product uses; with W_fa the sum over the feature's records
// touching block a of J_a^T J_f, the feature's share of S_ab is -Y_fa Y_fb^T with
// Y_fa = W_fa G_f (the block's rows x the feature's 3 or 4 coordinates).  One
// wavefront forms one block pair (a, b): each shared feature is one FP64 16x16x4
// MFMA (Y zero-padded to 16 x 4), and so is each record touching both a camera and a
// plane (U_ab = J_c^T J_g) and each relation between two groups; diagonal pairs add
// U_aa + lambda D_a.  Every pair sums in a fixed order, so S is the same run to run.
//
// Factorisation.  Right-looking blocked Cholesky on 64 x 64 tiles: one wavefront
// factors the diagonal tile and inverts its factor in LDS, the tiles below it become
// L_ik = A_ik L_kk^-T, and every trailing lower tile takes A_ij -= L_ik L_jk^T; both
// tile products are FP64 MFMA from LDS.  The triangular solves take one launch per
// tile column.  The matrix is padded to a multiple of 64 with identity rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "ba_internal.h"

namespace ba {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int NB = DENSE_NB;
constexpr int LDT = NB + 4;  // LDS row stride (doubles) of a tile in the tile products

inline unsigned nblk_dense(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// D += A B for one 16x16x4 FP64 MFMA.  Lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds D[l / 16 + 4 r][l % 16] in element r.
__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// first row of block b in A and its size
__device__ __forceinline__ void block_rows(const Dev& d, int b, int& o, int& n) {
  if (b < d.nc) { o = d.CD * b; n = d.CD; }
  else if (b < d.nc + d.ng) { o = d.offPl + 3 * (b - d.nc); n = 3; }
  else { o = d.offVp + 2 * (b - d.nc - d.ng); n = 2; }
}

template <int N> __device__ __forceinline__ int psym(int i, int j) {
  return i <= j ? i * N - i * (i - 1) / 2 + (j - i) : j * N - j * (j - 1) / 2 + (i - j);
}

// W += J_a^T J_f over the records of family FAM of feature f that touch block blk
template <int FAM, typename T, int CD>
__device__ __forceinline__ void acc_w(const Dev& d, int f, int blk, double (&W)[9][4]) {
  using F = Fam<FAM, CD>;
  using SL = Slot<FAM, CD>;
  const int kind = blk < d.nc ? 0 : blk < d.nc + d.ng ? 1 : 2;  // camera, plane, VP
  if (kind == 0 && F::NC == 0) return;
  if (kind != 0 && F::GT != kind) return;
  const int id = kind == 0 ? blk : kind == 1 ? blk - d.nc : blk - d.nc - d.ng;
  const int32_t* key = kind == 0 ? d.fcam[FAM] : d.fgrp[FAM];
  const int32_t r0 = d.foff[FAM][f], r1 = d.foff[FAM][f + 1];
  const T* base = (const T*)d.frec[FAM];
  for (int32_t r = r0; r < r1; ++r) {
    if (key[r] != id) continue;
    const T* s = base + (int64_t)r * SL::STRIDE;
    double jf[F::ROWS][F::NF];
#pragma unroll
    for (int row = 0; row < F::ROWS; ++row)
#pragma unroll
      for (int k = 0; k < F::NF; ++k) jf[row][k] = (double)s[SL::OF + row * F::NF + k];
    if (kind == 0) {
#pragma unroll
      for (int row = 0; row < F::ROWS; ++row)
#pragma unroll
        for (int i = 0; i < F::NC; ++i) {
          const double a = (double)s[SL::OC + row * F::NC + i];
#pragma unroll
          for (int k = 0; k < F::NF; ++k) W[i][k] += a * jf[row][k];
        }
    } else {
#pragma unroll
      for (int row = 0; row < F::ROWS; ++row)
#pragma unroll
        for (int i = 0; i < F::NG; ++i) {
          const double a = (double)s[SL::OG + row * F::NG + i];
#pragma unroll
          for (int k = 0; k < F::NF; ++k) W[i][k] += a * jf[row][k];
        }
    }
  }
}

// lower factor G of the feature's damped inverse V_f^-1 (the FP64 copy for blocks
// inverted in FP64); zero when that inverse is zero (failed FP64 Cholesky) or not
// positive definite
template <typename T, int NF> __device__ __forceinline__ void vinv_factor(const Dev& d, int f, double (&G)[4][4]) {
  constexpr int NS = NF * (NF + 1) / 2;
  const uint8_t fl = (NF == 3 ? d.flp : d.fll)[f];
  double M[NF][NF];
  if (fl) {
    const double* P = (NF == 3 ? d.Vip64 : d.Vil64) + (int64_t)NS * f;
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) M[i][j] = P[psym<NF>(i, j)];
  } else {
    const T* P = (const T*)(NF == 3 ? d.Vip : d.Vil) + (int64_t)NS * f;
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) M[i][j] = (double)P[psym<NF>(i, j)];
  }
  bool ok = true;
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    double s = M[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= G[j][k] * G[j][k];
    if (!(s > 0.0) || !isfinite(s)) ok = false;
    const double l = ok ? sqrt(s) : 1.0;
    G[j][j] = l;
#pragma unroll
    for (int i = j + 1; i < NF; ++i) {
      double t = M[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= G[i][k] * G[j][k];
      G[i][j] = t / l;
    }
  }
  if (!ok)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) G[i][j] = 0.0;
}

// Y of one (feature, block) entry, one thread per entry
template <typename T, int CD> __global__ __launch_bounds__(256) void k_dense_y(Dev d) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d.n_fent) return;
  const int2 fe = d.fent[e];
  const bool line = fe.x >= d.np;
  const int f = line ? fe.x - d.np : fe.x;
  double W[9][4], G[4][4];
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) W[i][k] = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) G[i][k] = 0.0;
  if (!line) {
    acc_w<1, T, CD>(d, f, fe.y, W);
    acc_w<3, T, CD>(d, f, fe.y, W);
    acc_w<6, T, CD>(d, f, fe.y, W);
    vinv_factor<T, 3>(d, f, G);
  } else {
    acc_w<2, T, CD>(d, f, fe.y, W);
    acc_w<4, T, CD>(d, f, fe.y, W);
    acc_w<5, T, CD>(d, f, fe.y, W);
    acc_w<7, T, CD>(d, f, fe.y, W);
    vinv_factor<T, 4>(d, f, G);
  }
  double* Y = d.dY + (int64_t)DENSE_Y * e;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      double y = 0.0;
#pragma unroll
      for (int m = 0; m < 4; ++m) y += W[i][m] * G[m][k];
      Y[k * 9 + i] = y;
    }
}

// S = 0 except the identity on the padding rows
__global__ __launch_bounds__(256) void k_dense_init(double* S, int n, int npad) {
  const int64_t tot = (int64_t)npad * npad;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / npad, c = i - r * npad;
    S[i] = (r == c && r >= n) ? 1.0 : 0.0;
  }
}

// one wavefront per block pair (a <= b): S_ab and, for a != b, S_ba = S_ab^T
template <typename T, int CD> __global__ __launch_bounds__(256) void k_dense_pair(Dev d, double lam) {
  const int p = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (p >= d.n_pair) return;
  const int lane = threadIdx.x & 63, i = lane & 15, k = lane >> 4;
  const int2 ab = d.pair_ab[p];
  const bool row = i < 9;
  const int yo = k * 9 + i;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  // shared features: -Y_fa Y_fb^T
  const int32_t e1 = d.pair_off[p + 1];
  int32_t e = d.pair_off[p];
  for (; e + 4 <= e1; e += 4) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int2 q = d.pair_ent[e + u];
      a[u] = row ? d.dY[(int64_t)DENSE_Y * q.x + yo] : 0.0;
      b[u] = row ? d.dY[(int64_t)DENSE_Y * q.y + yo] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = mfma16(-a[u], b[u], acc);
  }
  for (; e < e1; ++e) {
    const int2 q = d.pair_ent[e];
    const double a = row ? d.dY[(int64_t)DENSE_Y * q.x + yo] : 0.0;
    const double b = row ? d.dY[(int64_t)DENSE_Y * q.y + yo] : 0.0;
    acc = mfma16(-a, b, acc);
  }
  // U entries coupling two different blocks
  for (int32_t u = d.pair_uoff[p]; u < d.pair_uoff[p + 1]; ++u) {
    const int2 q = d.pair_u[u];
    double va = 0.0, vb = 0.0;
    if (q.x == 3) {
      using SL = Slot<3, CD>;
      const T* s = (const T*)d.frec[3] + (int64_t)q.y * SL::STRIDE;
      if (k < SL::ROWS && i < SL::NC) va = (double)s[SL::OC + k * SL::NC + i];
      if (k < SL::ROWS && i < SL::NG) vb = (double)s[SL::OG + k * SL::NG + i];
    } else if (q.x == 4) {
      using SL = Slot<4, CD>;
      const T* s = (const T*)d.frec[4] + (int64_t)q.y * SL::STRIDE;
      if (k < SL::ROWS && i < SL::NC) va = (double)s[SL::OC + k * SL::NC + i];
      if (k < SL::ROWS && i < SL::NG) vb = (double)s[SL::OG + k * SL::NG + i];
    } else {
      // relation: 3 rows of [J_a (3) | J_b (3)]; code 8: a is the relation's first group
      const double* J = d.rel_J + (int64_t)q.y * 18;
      const int ca = q.x == 8 ? 0 : 3, cb = 3 - ca;
      if (k < 3 && i < 3) {
        va = J[k * 6 + ca + i];
        vb = J[k * 6 + cb + i];
      }
    }
    acc = mfma16(va, vb, acc);
  }
  int oa, na, ob, nb;
  block_rows(d, ab.x, oa, na);
  block_rows(d, ab.y, ob, nb);
  const int64_t ld = d.dense_npad;
  const int j = lane & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ii = k + 4 * r;
    if (ii < na && j < nb) {
      double v = acc[r];
      if (ab.x == ab.y) {
        const int b = ab.x;
        if (b < d.nc) v += d.Ucam[(int64_t)b * d.CD * d.CD + ii * d.CD + j];
        else if (b < d.nc + d.ng) v += d.Upl[9 * (int64_t)(b - d.nc) + 3 * ii + j];
        else v += d.Uvp[4 * (int64_t)(b - d.nc - d.ng) + 2 * ii + j];
        if (ii == j) v += lam * d.DA[oa + ii];
        d.dS[(oa + ii) * ld + ob + j] = v;
      } else {
        d.dS[(oa + ii) * ld + ob + j] = v;
        d.dS[(ob + j) * ld + oa + ii] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// blocked Cholesky

// diagonal tile k: L_kk (lower, in place; the upper part is zeroed) and L_kk^-1
// into Linv; *info = 1 + the global column of the first non-positive pivot.  One
// wavefront; lane t owns row t while factoring and column t while inverting.
__global__ __launch_bounds__(64) void k_chol_diag(double* A, int ld, int k, double* Linv, int* info) {
  if (*info) return;
  __shared__ double L[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  const int t = threadIdx.x;
  double* Akk = A + (int64_t)NB * k * ld + (int64_t)NB * k;
  for (int r = 0; r < NB; ++r) L[r][t] = Akk[(int64_t)r * ld + t];
  __syncthreads();
  for (int j = 0; j < NB; ++j) {
    double s = 0.0;
    if (t >= j) {
      s = L[t][j];
      for (int m = 0; m < j; ++m) s -= L[t][m] * L[j][m];
    }
    const double piv = __shfl(s, j, 64);
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (t == 0) *info = NB * k + j + 1;
      return;
    }
    const double ljj = sqrt(piv);
    if (t >= j) L[t][j] = t == j ? ljj : s / ljj;
    __syncthreads();
  }
  for (int r = 0; r < NB; ++r) {
    if (r >= t) {
      double s = r == t ? 1.0 : 0.0;
      for (int m = t; m < r; ++m) s -= L[r][m] * X[m][t];
      X[r][t] = s / L[r][r];
    }
  }
  __syncthreads();
  double* Li = Linv + (int64_t)k * NB * NB;
  for (int r = 0; r < NB; ++r) {
    Akk[(int64_t)r * ld + t] = t <= r ? L[r][t] : 0.0;
    Li[r * NB + t] = t <= r ? X[r][t] : 0.0;
  }
}

__device__ __forceinline__ void load_tile(double (*S)[LDT], const double* src, int64_t ld) {
  const int t = threadIdx.x;
#pragma unroll 4
  for (int q = 0; q < NB / 4; ++q) {
    const int r = 4 * q + (t >> 6), c = t & 63;
    S[r][c] = src[r * ld + c];
  }
}

// acc[jt] = (As Bs^T) for rows 16 w .. 16 w + 15 and columns 16 jt .. 16 jt + 15 (w: wavefront)
__device__ __forceinline__ void gemm_nt(const double (*As)[LDT], const double (*Bs)[LDT], v4d (&acc)[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int jt = 0; jt < 4; ++jt) acc[jt] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int kk = 0; kk < NB / 4; ++kk) {
    const double a = As[16 * w + i][4 * kk + kq];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) acc[jt] = mfma16(a, Bs[16 * jt + i][4 * kk + kq], acc[jt]);
  }
}

// the tiles below diagonal tile k: L_ik = A_ik L_kk^-T
__global__ __launch_bounds__(256) void k_chol_panel(double* A, int ld, int k, const double* Linv, const int* info) {
  if (*info) return;
  __shared__ double As[NB][LDT], Bs[NB][LDT];
  const int I = k + 1 + blockIdx.x;
  double* Aik = A + (int64_t)NB * I * ld + (int64_t)NB * k;
  load_tile(As, Aik, ld);
  load_tile(Bs, Linv + (int64_t)k * NB * NB, NB);
  __syncthreads();
  v4d acc[4];
  gemm_nt(As, Bs, acc);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int jt = 0; jt < 4; ++jt)
#pragma unroll
    for (int r = 0; r < 4; ++r) Aik[(int64_t)(16 * w + (lane >> 4) + 4 * r) * ld + 16 * jt + (lane & 15)] = acc[jt][r];
}

// trailing lower tiles (I, J), k < J <= I: A_IJ -= L_Ik L_Jk^T; blockIdx = I' (I' + 1) / 2 + J'
__global__ __launch_bounds__(256) void k_chol_update(double* A, int ld, int k, const int* info) {
  if (*info) return;
  __shared__ double As[NB][LDT], Bs[NB][LDT];
  const int idx = blockIdx.x;
  int ii = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
  while ((ii + 1) * (ii + 2) / 2 <= idx) ++ii;
  while (ii * (ii + 1) / 2 > idx) --ii;
  const int jj = idx - ii * (ii + 1) / 2;
  const int I = k + 1 + ii, J = k + 1 + jj;
  load_tile(As, A + (int64_t)NB * I * ld + (int64_t)NB * k, ld);
  load_tile(Bs, A + (int64_t)NB * J * ld + (int64_t)NB * k, ld);
  __syncthreads();
  v4d acc[4];
  gemm_nt(As, Bs, acc);
  double* C = A + (int64_t)NB * I * ld + (int64_t)NB * J;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int jt = 0; jt < 4; ++jt)
#pragma unroll
    for (int r = 0; r < 4; ++r) C[(int64_t)(16 * w + (lane >> 4) + 4 * r) * ld + 16 * jt + (lane & 15)] -= acc[jt][r];
}

// forward solve, tile column k: y_k = L_kk^-1 v_k into w (workgroup 0); the others
// (I = k + workgroup) take v_I -= L_Ik y_k
__global__ __launch_bounds__(64) void k_trsv_fwd(const double* A, int ld, int k, const double* Linv, double* v, double* w,
                                                  const int* info) {
  if (*info) return;
  __shared__ double bk[NB], yk[NB];
  __shared__ double Ls[NB][NB + 1];
  const int t = threadIdx.x, I = k + blockIdx.x;
  bk[t] = v[NB * k + t];
  __syncthreads();
  const double* Li = Linv + (int64_t)k * NB * NB;
  double y = 0.0;
  for (int m = 0; m <= t; ++m) y += Li[t * NB + m] * bk[m];
  if (blockIdx.x == 0) {
    w[NB * k + t] = y;
    return;
  }
  yk[t] = y;
  const double* Lik = A + (int64_t)NB * I * ld + (int64_t)NB * k;
  for (int r = 0; r < NB; ++r) Ls[r][t] = Lik[(int64_t)r * ld + t];
  __syncthreads();
  double s = 0.0;
  for (int c = 0; c < NB; ++c) s += Ls[t][c] * yk[c];
  v[NB * I + t] -= s;
}

// backward solve, tile column k (descending): x_k = L_kk^-T w_k into v (workgroup 0);
// the others (J = k - workgroup) take w_J -= L_kJ^T x_k
__global__ __launch_bounds__(64) void k_trsv_bwd(const double* A, int ld, int k, const double* Linv, double* v, double* w,
                                                  const int* info) {
  if (*info) return;
  __shared__ double yk[NB], xk[NB];
  const int t = threadIdx.x, J = k - blockIdx.x;
  yk[t] = w[NB * k + t];
  __syncthreads();
  const double* Li = Linv + (int64_t)k * NB * NB;
  double x = 0.0;
  for (int r = t; r < NB; ++r) x += Li[r * NB + t] * yk[r];
  if (blockIdx.x == 0) {
    v[NB * k + t] = x;
    return;
  }
  xk[t] = x;
  __syncthreads();
  double s = 0.0;
  for (int r = 0; r < NB; ++r) s += A[(int64_t)(NB * k + r) * ld + (int64_t)NB * J + t] * xk[r];
  w[NB * J + t] -= s;
}

__global__ void k_zero_upper(double* A, int npad) {
  const int64_t tot = (int64_t)npad * npad;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x)
    if (i % npad > i / npad) A[i] = 0.0;
}

__global__ void k_dense_rhs(double* v, const double* b, int n, int npad) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npad; i += gridDim.x * blockDim.x) v[i] = i < n ? b[i] : 0.0;
}

__global__ void k_dense_out(double* x, const double* v, int n, const int* info) {
  if (*info) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] = v[i];
}

// |S x - b|^2 and |b|^2 (S x in q, from the implicit product) into the PCG scalars,
// which then describe the direct solve: no iterations, done, no breakdown
__global__ __launch_bounds__(1024) void k_dense_resid(Dev d) {
  __shared__ double lds[2][16];
  double rr = 0.0, bb = 0.0;
  for (int i = threadIdx.x; i < d.nA; i += blockDim.x) {
    const double r = d.q[i] - d.bA[i];
    rr += r * r;
    bb += d.bA[i] * d.bA[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    rr += __shfl_xor(rr, o, 64);
    bb += __shfl_xor(bb, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    lds[0][threadIdx.x >> 6] = rr;
    lds[1][threadIdx.x >> 6] = bb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { a += lds[0][w]; b += lds[1][w]; }
    d.scal[SC_RR] = a;
    d.scal[SC_BB] = b;
    d.scal[SC_ITER] = 0;
    d.scal[SC_DONE] = 1;
    d.scal[SC_BREAK] = 0;
    d.scal[SC_COARSE] = 0;
  }
}

}  // namespace

void launch_dense_assemble(const Dev& d, double lambda, hipStream_t s) {
  if (d.dense_n == 0) return;
  const int64_t tot = (int64_t)d.dense_npad * d.dense_npad;
  k_dense_init<<<(unsigned)std::min<int64_t>(nblk_dense(tot, 256), 8192), 256, 0, s>>>(d.dS, d.dense_n, d.dense_npad);
  BA_DISPATCH_T_CD(d, {
    if (d.n_fent) k_dense_y<T, CD><<<nblk_dense(d.n_fent, 256), 256, 0, s>>>(d);
    if (d.n_pair) k_dense_pair<T, CD><<<nblk_dense(d.n_pair, 4), 256, 0, s>>>(d, lambda);
  });
}

void launch_dense_factor_solve(double* A, int npad, double* Linv, double* v, double* w, int* info, hipStream_t s) {
  const int nt = npad / NB;
  for (int k = 0; k < nt; ++k) {
    k_chol_diag<<<1, 64, 0, s>>>(A, npad, k, Linv, info);
    const int m = nt - k - 1;
    if (m > 0) {
      k_chol_panel<<<m, 256, 0, s>>>(A, npad, k, Linv, info);
      k_chol_update<<<m * (m + 1) / 2, 256, 0, s>>>(A, npad, k, info);
    }
  }
  for (int k = 0; k < nt; ++k) k_trsv_fwd<<<nt - k, 64, 0, s>>>(A, npad, k, Linv, v, w, info);
  for (int k = nt - 1; k >= 0; --k) k_trsv_bwd<<<k + 1, 64, 0, s>>>(A, npad, k, Linv, v, w, info);
}

void launch_dense_solve(const Dev& d, double lambda, hipStream_t s) {
  launch_zero(d.dinfo, sizeof(int), s);
  if (d.dense_n == 0) return;
  launch_dense_assemble(d, lambda, s);
  k_dense_rhs<<<nblk_dense(d.dense_npad, 256), 256, 0, s>>>(d.dv, d.bA, d.dense_n, d.dense_npad);
  launch_dense_factor_solve(d.dS, d.dense_npad, d.dLinv, d.dv, d.dw, d.dinfo, s);
  k_dense_out<<<nblk_dense(d.dense_n, 256), 256, 0, s>>>(d.x, d.dv, d.dense_n, d.dinfo);
}

void launch_dense_residual(const Dev& d, double lambda, hipStream_t s) {
  if (d.nA == 0) return;
  launch_schur_matvec(d, d.x, d.q, lambda, s);
  k_dense_resid<<<1, 1024, 0, s>>>(d);
}

void launch_dense_pad_identity(double* A, int n, int npad, hipStream_t s) {
  const int64_t tot = (int64_t)npad * npad;
  if (tot) k_dense_init<<<(unsigned)std::min<int64_t>(nblk_dense(tot, 256), 8192), 256, 0, s>>>(A, n, npad);
}

void launch_dense_zero_upper(double* A, int npad, hipStream_t s) {
  const int64_t tot = (int64_t)npad * npad;
  if (tot) k_zero_upper<<<(unsigned)std::min<int64_t>(nblk_dense(tot, 256), 8192), 256, 0, s>>>(A, npad);
}

}  // namespace ba
