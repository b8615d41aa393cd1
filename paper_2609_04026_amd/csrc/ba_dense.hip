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
// tile products are FP64 MFMA from LDS.  The forward solve rides along (diagonal tile:
// y_k = L_kk^-1 v_k; tiles below: v_i -= L_ik y_k); the backward solve takes one launch
// per tile column.  The matrix is padded to a multiple of 64 with identity rows.
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
    acc_w<8, T, CD>(d, f, fe.y, W);
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

// Consecutive workgroups go to different XCDs: workgroup g works on item group
// (g % 8) * per + g / 8, so that each XCD takes a contiguous run of block pairs
// (pairs are sorted by (a, b): a run shares the Y of block a in that XCD's L2).
// Launched with 8 * per workgroups; a workgroup past the end returns.
__device__ __forceinline__ int xcd_group(int per) { return (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8); }

// sum over the shared-feature entries [e, e1) of -Y_fa Y_fb^T (the wavefront's MFMA
// accumulator; lanes with i >= 9 contribute zero rows / columns)
__device__ __forceinline__ v4d feature_terms(const Dev& d, int32_t e, int32_t e1, int lane) {
  const int i = lane & 15, k = lane >> 4;
  const bool row = i < 9;
  const int yo = k * 9 + i;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (; e + 8 <= e1; e += 8) {
    int2 q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) q[u] = d.pair_ent[e + u];
    double a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = row ? d.dY[(int64_t)DENSE_Y * q[u].x + yo] : 0.0;
      b[u] = row ? d.dY[(int64_t)DENSE_Y * q[u].y + yo] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = mfma16(-a[u], b[u], acc);
  }
  for (; e < e1; ++e) {
    const int2 q = d.pair_ent[e];
    const double a = row ? d.dY[(int64_t)DENSE_Y * q.x + yo] : 0.0;
    const double b = row ? d.dY[(int64_t)DENSE_Y * q.y + yo] : 0.0;
    acc = mfma16(-a, b, acc);
  }
  return acc;
}

// one wavefront per chunk of a pair with many shared features: its partial sum, rows
// 0 .. 11 of the accumulator (elements 0 .. 2) stored lane-major
__global__ __launch_bounds__(256) void k_dense_chunk(Dev d, int per) {
  const int c = 4 * xcd_group(per) + (int)(threadIdx.x >> 6);
  if (c >= d.n_chunk) return;
  const int lane = threadIdx.x & 63;
  const int2 rg = d.chunk[c];
  const v4d acc = feature_terms(d, rg.x, rg.y, lane);
#pragma unroll
  for (int r = 0; r < 3; ++r) d.dpart[((int64_t)c * 3 + r) * 64 + lane] = acc[r];
}

// one wavefront per block pair (a <= b): S_ab and, for a != b, S_ba = S_ab^T; the
// shared features summed here, or (pairs with chunks) their chunks' partials in order
template <typename T, int CD> __global__ __launch_bounds__(256) void k_dense_pair(Dev d, double lam, int per) {
  const int p = 4 * xcd_group(per) + (int)(threadIdx.x >> 6);
  if (p >= d.n_pair) return;
  const int lane = threadIdx.x & 63, i = lane & 15, k = lane >> 4;
  const int2 ab = d.pair_ab[p];
  v4d acc;
  const int32_t c0 = d.pair_choff[p], c1 = d.pair_choff[p + 1];
  if (c0 == c1) {
    acc = feature_terms(d, d.pair_off[p], d.pair_off[p + 1], lane);
  } else {
    acc = v4d{0.0, 0.0, 0.0, 0.0};
    for (int32_t c = c0; c < c1; ++c)
#pragma unroll
      for (int r = 0; r < 3; ++r) acc[r] += d.dpart[((int64_t)c * 3 + r) * 64 + lane];
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
// blocked Cholesky, with the forward solve L y = v folded into the factorisation
// (diagonal tile k: y_k = L_kk^-1 v_k; tile below it: v_i -= L_ik y_k)

// diagonal tile k: L_kk (lower, in place; the upper part zeroed), L_kk^-1 into Linv,
// y_k = L_kk^-1 v_k into w; *info = 1 + the global column of the first non-positive
// pivot.  Block LDL^T elimination in steps of 4 columns, with the identity carried
// along so that the same steps yield the inverse: at step J the 4 x 4 block D_J (the
// Schur complement of the earlier columns) is factored D_J = L_D L_D^T in every lane
// (W = L_D^-1), row t's multipliers are u_t = D_J^-1 r_t (r_t: its entries in the
// block's columns), and every later row takes row_t -= u_t . [block rows] on its
// columns and on its carried identity part.  Then L[t][block] = W r_t, and L^-1 is
// W_J applied to the carried rows of block J.  Four wavefronts; lane t of wavefront h
// holds columns 16 h .. 16 h + 15 of row t in registers (the steps within one
// wavefront's columns are unrolled, so register indices are static); one barrier per
// step (LDS broadcasts double-buffered).
__global__ __launch_bounds__(256) void k_chol_diag(double* A, int ld, int k, double* Linv, const double* v, double* w,
                                                   int* info) {
  if (*info) return;
  __shared__ double Ls[NB][NB + 1];
  __shared__ double bufA[2][NB][4];
  __shared__ double bufX[2][4][NB];
  __shared__ double Wd[NB / 4][4][4];
  __shared__ double vk[NB];
  __shared__ double red[4][NB];
  const int t = threadIdx.x & 63, h = threadIdx.x >> 6;
  double* Akk = A + (int64_t)NB * k * ld + (int64_t)NB * k;
  if (h == 0) vk[t] = v[NB * k + t];
#pragma unroll
  for (int q = 0; q < NB / 4; ++q) Ls[4 * q + h][t] = Akk[(int64_t)(4 * q + h) * ld + t];
  __syncthreads();
  double a[16], x[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    a[c] = Ls[t][16 * h + c];
    x[c] = 16 * h + c == t ? 1.0 : 0.0;
  }
  // outer loop not unrolled: the fully unrolled kernel (90 KB) overflows the 64 KB
  // instruction cache, and a launch runs it once
#pragma unroll 1
  for (int hj = 0; hj < 4; ++hj)
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    const int J = 4 * hj + jj, o = 4 * jj, j0 = 4 * J;
    double (*bA)[4] = bufA[J & 1];
    double (*bX)[NB] = bufX[J & 1];
    if (h == hj)
#pragma unroll
      for (int q = 0; q < 4; ++q) bA[t][q] = a[o + q];
    if ((t >> 2) == J)
#pragma unroll
      for (int c = 0; c < 16; ++c) bX[t & 3][16 * h + c] = x[c];
    __syncthreads();
    // D_J = L_D L_D^T and W = L_D^-1, the same in every lane
    double Ld[4][4], W[4][4];
    int fail = -1;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        Ld[i][q] = i >= q ? bA[j0 + i][q] : 0.0;
        W[i][q] = 0.0;
      }
    // one reciprocal square root per pivot and no divisions: the 4 x 4 factorisation
    // is the serial part of every step
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double sj = Ld[j][j];
#pragma unroll
      for (int m = 0; m < j; ++m) sj -= Ld[j][m] * Ld[j][m];
      if ((!(sj > 0.0) || !isfinite(sj)) && fail < 0) fail = j;
      const double rj = rsqrt(fmax(sj, 1e-300));
      Ld[j][j] = sj * rj;
      W[j][j] = rj;
#pragma unroll
      for (int i = j + 1; i < 4; ++i) {
        double si = Ld[i][j];
#pragma unroll
        for (int m = 0; m < j; ++m) si -= Ld[i][m] * Ld[j][m];
        Ld[i][j] = si * rj;
      }
    }
    if (fail >= 0) {
      if (threadIdx.x == 0) *info = NB * k + j0 + fail + 1;
      return;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = j + 1; i < 4; ++i) {
        double si = 0.0;
#pragma unroll
        for (int m = j; m < i; ++m) si -= Ld[i][m] * W[m][j];
        W[i][j] = si * W[i][i];
      }
    if (threadIdx.x == 0)
#pragma unroll
      for (int q = 0; q < 16; ++q) Wd[J][q >> 2][q & 3] = W[q >> 2][q & 3];
    double r[4], l[4], u[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = bA[t][q];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      l[q] = 0.0;
#pragma unroll
      for (int p = 0; p <= q; ++p) l[q] += W[q][p] * r[p];
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      u[p] = 0.0;
#pragma unroll
      for (int q = p; q < 4; ++q) u[p] += l[q] * W[q][p];
    }
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (16 * h + c >= j0 + 4) {
        const double* rc = bA[16 * h + c];
        a[c] -= u[0] * rc[0] + u[1] * rc[1] + u[2] * rc[2] + u[3] * rc[3];
      }
    if (t >= j0 + 4) {
#pragma unroll
      for (int c = 0; c < 16; ++c)
        x[c] -= u[0] * bX[0][16 * h + c] + u[1] * bX[1][16 * h + c] + u[2] * bX[2][16 * h + c] +
                u[3] * bX[3][16 * h + c];
    }
    if (h == hj) {
      if (t >= j0 + 4) {
#pragma unroll
        for (int q = 0; q < 4; ++q) a[o + q] = l[q];
      } else if ((t >> 2) == J) {
        const int i = t & 3;
#pragma unroll
        for (int q = 0; q < 4; ++q) a[o + q] = i == 0 ? Ld[0][q] : i == 1 ? Ld[1][q] : i == 2 ? Ld[2][q] : Ld[3][q];
      }
    }
  }
  // L (zero upper part) back to the tile; the carried rows to LDS for L^-1
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    Akk[(int64_t)t * ld + 16 * h + c] = 16 * h + c <= t ? a[c] : 0.0;
    Ls[t][16 * h + c] = x[c];
  }
  __syncthreads();
  double* Li = Linv + (int64_t)k * NB * NB;
  const int J = t >> 2, i = t & 3;
  double y = 0.0;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    double xs = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) xs += Wd[J][i][q] * Ls[4 * J + q][16 * h + c];
    Li[t * NB + 16 * h + c] = xs;
    y += xs * vk[16 * h + c];
  }
  red[h][t] = y;
  __syncthreads();
  if (h == 0) w[NB * k + t] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
}

__device__ __forceinline__ void load_tile(double (*S)[LDT], const double* src, int64_t ld) {
  const int t = threadIdx.x;
#pragma unroll
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

// the tiles below diagonal tile k: L_ik = A_ik L_kk^-T, then v_i -= L_ik y_k
__global__ __launch_bounds__(256) void k_chol_panel(double* A, int ld, int k, const double* Linv, double* v,
                                                    const double* w, const int* info) {
  if (*info) return;
  __shared__ double As[NB][LDT], Bs[NB][LDT];
  __shared__ double yk[NB];
  const int t = threadIdx.x;
  const int I = k + 1 + blockIdx.x;
  double* Aik = A + (int64_t)NB * I * ld + (int64_t)NB * k;
  if (t < NB) yk[t] = w[NB * k + t];
  load_tile(As, Aik, ld);
  load_tile(Bs, Linv + (int64_t)k * NB * NB, NB);
  __syncthreads();
  v4d acc[4];
  gemm_nt(As, Bs, acc);
  const int lane = t & 63, wv = t >> 6;
  __syncthreads();
#pragma unroll
  for (int jt = 0; jt < 4; ++jt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * wv + (lane >> 4) + 4 * r, c = 16 * jt + (lane & 15);
      Aik[(int64_t)row * ld + c] = acc[jt][r];
      As[row][c] = acc[jt][r];
    }
  __syncthreads();
  const int row = t >> 2, part = t & 3;
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < 16; ++m) s += As[row][16 * part + m] * yk[16 * part + m];
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  if (part == 0) v[NB * I + row] -= s;
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

// backward solve, tile column k (descending): x_k = L_kk^-T w_k into v (workgroup 0);
// the others (J = k - workgroup) take w_J -= L_kJ^T x_k.  Thread (c, part) sums rows
// 16 part .. 16 part + 15 of column c.
__global__ __launch_bounds__(256) void k_trsv_bwd(const double* A, int ld, int k, const double* Linv, double* v, double* w,
                                                  const int* info) {
  if (*info) return;
  __shared__ double yk[NB], xk[NB];
  __shared__ double red[4][NB];
  const int t = threadIdx.x, c = t & 63, part = t >> 6, J = k - blockIdx.x;
  if (t < NB) yk[t] = w[NB * k + t];
  __syncthreads();
  const double* Li = Linv + (int64_t)k * NB * NB;
  double x = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) x += Li[(16 * part + q) * NB + c] * yk[16 * part + q];
  red[part][c] = x;
  __syncthreads();
  x = red[0][c] + red[1][c] + red[2][c] + red[3][c];
  if (blockIdx.x == 0) {
    if (t < NB) v[NB * k + t] = x;
    return;
  }
  if (t < NB) xk[t] = x;
  __syncthreads();
  const double* Lk = A + (int64_t)NB * k * ld + (int64_t)NB * J;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) s += Lk[(int64_t)(16 * part + q) * ld + c] * xk[16 * part + q];
  red[part][c] = s;
  __syncthreads();
  if (t < NB) w[NB * J + t] -= red[0][t] + red[1][t] + red[2][t] + red[3][t];
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
    if (d.n_chunk) {
    const int per = (int)nblk_dense(nblk_dense(d.n_chunk, 4), 8);
    k_dense_chunk<<<8 * per, 256, 0, s>>>(d, per);
  }
  if (d.n_pair) {
    const int per = (int)nblk_dense(nblk_dense(d.n_pair, 4), 8);
    k_dense_pair<T, CD><<<8 * per, 256, 0, s>>>(d, lambda, per);
  }
  });
}

void launch_dense_factor_solve(double* A, int npad, double* Linv, double* v, double* w, int* info, hipStream_t s) {
  const int nt = npad / NB;
  for (int k = 0; k < nt; ++k) {
    k_chol_diag<<<1, 256, 0, s>>>(A, npad, k, Linv, v, w, info);
    const int m = nt - k - 1;
    if (m > 0) {
      k_chol_panel<<<m, 256, 0, s>>>(A, npad, k, Linv, v, w, info);
      k_chol_update<<<m * (m + 1) / 2, 256, 0, s>>>(A, npad, k, info);
    }
  }
  for (int k = nt - 1; k >= 0; --k) k_trsv_bwd<<<k + 1, 256, 0, s>>>(A, npad, k, Linv, v, w, info);
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
