// HIP kernels of one LM iteration of holistic bundle adjustment on gfx950.
//
// Pass structure (all on one stream):
//   cast      FP64 master parameters -> work copy in T
//   linearize one lane per record: IRLS-weighted residual (from FP64
//             parameters) and analytic Jacobian (in T) -> AoS record slots
//   feature   one lane per feature: V_f = sum J_f^T J_f, g_f; damping; FP32
//             Cholesky with a condition test, FP64 redo of flagged blocks
//   camera    one workgroup per camera (group): U_aa, g_a, and per lambda the
//             damped diagonal blocks of S and b with pair-summed W_af
//   pcg       implicit-Schur product: wavefront tiles of whole features, one
//             record per lane: J_a x, the feature sums by a segmented scan,
//             V_f^-1 on the feature's last lane, then J_a^T accumulated into a
//             workgroup-private copy of the reduced vector in LDS; features too
//             large for a tile one wavefront each; FP64 vector updates and dots
//   backsub   the same tiles (and one wavefront per large feature): h_f and the
//             model decrease terms
//   cost      one lane per record: FP64 residuals and robust cost
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>

#include "ba_internal.h"

namespace ba {

// ---------------------------------------------------------------------------
// shape helpers visible to the host
int slot_stride(int fam, int cd) {
#define SS(F) (cd == 9 ? Slot<F, 9>::STRIDE : Slot<F, 6>::STRIDE)
  switch (fam) {
    case 1: return SS(1); case 2: return SS(2); case 3: return SS(3); case 4: return SS(4);
    case 5: return SS(5); case 6: return SS(6); case 7: return SS(7); case 8: return SS(8);
    case 9: return SS(9); case 10: return SS(10);
  }
#undef SS
  return 0;
}
int slot_nc(int fam, int cd) {
  switch (fam) {
    case 1: case 3: case 6: case 9: return cd;
    case 2: case 4: case 7: case 10: return cd == 9 ? 7 : 6;
  }
  return 0;
}
int slot_ng(int fam) { return fam == 3 || fam == 4 || fam == 8 ? 3 : fam == 5 ? 2 : fam == 9 || fam == 10 ? SH_DOF : 0; }
int slot_nf(int fam) { return fam_is_line(fam) ? 4 : 3; }


static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------------------
// small device helpers
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Sum K values over a workgroup.  lds must hold (nwaves + 1) * K elements.
// Results are returned in lds[nwaves * K + k] (valid after the call for all threads).
template <typename T, int K> __device__ __forceinline__ T* block_sum_arr(T (&v)[K], T* lds) {
  const int nw = (blockDim.x + 63) >> 6, w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (l == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[w * K + k] = v[k];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    T s = 0;
    for (int i = 0; i < nw; ++i) s += lds[i * K + k];
    lds[nw * K + k] = s;
  }
  __syncthreads();
  return lds + nw * K;
}

template <typename T, int N> __device__ __forceinline__ void load_vec(const T* __restrict__ p, T (&v)[N]) {
  static_assert(N % 4 == 0, "slot stride must be a multiple of 4");
  if constexpr (sizeof(T) == 4) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      float4 a = q[i];
      v[4 * i] = a.x; v[4 * i + 1] = a.y; v[4 * i + 2] = a.z; v[4 * i + 3] = a.w;
    }
  } else {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      double2 a = q[i];
      v[2 * i] = a.x; v[2 * i + 1] = a.y;
    }
  }
}

template <typename T, int N> __device__ __forceinline__ void store_vec(T* __restrict__ p, const T (&v)[N]) {
  if constexpr (sizeof(T) == 4) {
    float4* q = reinterpret_cast<float4*>(p);
#pragma unroll
    for (int i = 0; i < N / 4; ++i) q[i] = make_float4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);
  } else {
    double2* q = reinterpret_cast<double2*>(p);
#pragma unroll
    for (int i = 0; i < N / 2; ++i) q[i] = make_double2(v[2 * i], v[2 * i + 1]);
  }
}

// packed symmetric index (i <= j) of an N x N matrix
template <int N> __host__ __device__ constexpr int sym(int i, int j) {
  return i <= j ? i * N - i * (i - 1) / 2 + (j - i) : j * N - j * (j - 1) / 2 + (i - j);
}

// Cholesky of a full N x N SPD matrix (lower factor in place).  Returns false
// on a non-positive or non-finite pivot.
template <typename S, int N> __device__ __forceinline__ bool chol(S (&A)[N][N]) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    S s = A[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= A[j][k] * A[j][k];
    if (!(s > S(0)) || !isfinite(s)) return false;
    S ljj = sqrt(s);
    A[j][j] = ljj;
    S inv = S(1) / ljj;
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      S t = A[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= A[i][k] * A[j][k];
      A[i][j] = t * inv;
    }
  }
  return true;
}

// inverse of A = L L^T from its lower Cholesky factor (full output)
template <typename S, int N> __device__ __forceinline__ void chol_inverse(const S (&L)[N][N], S (&Ai)[N][N]) {
  S Li[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) Li[i][j] = 0;
  }
#pragma unroll
  for (int j = 0; j < N; ++j) {
    Li[j][j] = S(1) / L[j][j];
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      S t = 0;
#pragma unroll
      for (int k = j; k < i; ++k) t -= L[i][k] * Li[k][j];
      Li[i][j] = t / L[i][i];
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      S t = 0;
#pragma unroll
      for (int k = (i > j ? i : j); k < N; ++k) t += Li[k][i] * Li[k][j];
      Ai[i][j] = t;
    }
  }
}


// ---------------------------------------------------------------------------
// parameter cast
template <typename T> __global__ void k_cast(Dev d, int candidate) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nthr = (int64_t)gridDim.x * blockDim.x;
  auto cp = [&](const double* s, void* dv, int64_t n) {
    T* dst = (T*)dv;
    for (int64_t i = tid; i < n; i += nthr) dst[i] = (T)s[i];
  };
  cp(candidate ? d.cam64n : d.cam64, d.camT, (int64_t)d.nc * CAM_STRIDE);
  cp(candidate ? d.pt64n : d.pt64, d.ptT, (int64_t)d.np * PT_STRIDE);
  cp(candidate ? d.ln64n : d.ln64, d.lnT, (int64_t)d.nl * LN_STRIDE);
  cp(candidate ? d.pl64n : d.pl64, d.plT, (int64_t)d.ng * PL_STRIDE);
  cp(candidate ? d.vp64n : d.vp64, d.vpT, (int64_t)d.nv * VP_STRIDE);
}

void launch_cast_params(const Dev& d, bool candidate, hipStream_t s) {
  if (d.fp64) k_cast<double><<<256, 256, 0, s>>>(d, candidate ? 1 : 0);
  else k_cast<float><<<256, 256, 0, s>>>(d, candidate ? 1 : 0);
}

// ---------------------------------------------------------------------------
// FP64 residual of one record (shared by linearisation and cost)
template <int FAM> __device__ __forceinline__ void residual64(const Dev& d, int64_t i, const double* cam, const double* pt,
                                                              const double* ln, const double* pl, const double* vp,
                                                              const double* sh, double* r) {
  using F = Fam<FAM, 9>;
  const int f = d.ffeat[FAM][i];
  double m[4] = {0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < F::MEAS; ++k) m[k] = d.fmeas[FAM][i * F::MEAS + k];
  if constexpr (FAM == 5) {
    const int g = d.fgrp[FAM][i];
    res_R5<double>(load_line<double>(ln + (int64_t)LN_STRIDE * f), load_vp<double>(vp + (int64_t)VP_STRIDE * g), r);
  } else if constexpr (FAM == 8) {
    res_R12<double>(pt + (int64_t)PT_STRIDE * f, load_plane<double>(pl + (int64_t)PL_STRIDE * d.fgrp[FAM][i]), r);
  } else {
    const int c = d.fcam[FAM][i];
    Cam<double> C = load_cam<double>(cam + (int64_t)CAM_STRIDE * c);
    if constexpr (FAM == 1 || FAM == 3 || FAM == 6 || FAM == 9) {
      const double* X = pt + (int64_t)PT_STRIDE * f;
      if constexpr (FAM == 1) res_R1<double>(C, X, m, r);
      if constexpr (FAM == 3) res_R3<double>(C, X, load_plane<double>(pl + (int64_t)PL_STRIDE * d.fgrp[FAM][i]), r);
      if constexpr (FAM == 6) res_R6<double>(C, X, m, r);
      if constexpr (FAM == 9) {
        const double* S = sh + (int64_t)SH_STRIDE * d.fgrp[FAM][i];
        res_R13<double>(C, X, S, shape_type(S) == SH_CUBOID ? cuboid_face<double>(S, X) : 0, r);
      }
    } else {
      Line<double> L = load_line<double>(ln + (int64_t)LN_STRIDE * f);
      if constexpr (FAM == 2) res_R2<double>(C, L, m, r);
      if constexpr (FAM == 4) res_R4<double>(C, L, load_plane<double>(pl + (int64_t)PL_STRIDE * d.fgrp[FAM][i]), m, r);
      if constexpr (FAM == 7) res_R7<double>(C, L, m, r);
      if constexpr (FAM == 10) {
        const double* S = sh + (int64_t)SH_STRIDE * d.fgrp[FAM][i];
        double dl[3], ml[3];
        line_dm(L, dl, ml);
        res_R14<double>(C, L, S, cuboid_face_line<double>(S, dl, ml), m, r);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// relative image-line normal of a line-projection record, from the FP64 master
// parameters (for R4 the smaller of the line's and of its plane projection's)
template <int FAM> __device__ __forceinline__ double line_record_normal(const Dev& d, int64_t i, int f) {
  const Cam<double> C = load_cam<double>(d.cam64 + (int64_t)CAM_STRIDE * d.fcam[FAM][i]);
  const Line<double> L = load_line<double>(d.ln64 + (int64_t)LN_STRIDE * f);
  double dl[3], ml[3];
  line_dm(L, dl, ml);
  double rel = image_line_normal(C, dl, ml);
  if constexpr (FAM == 4) {
    PlaneLine<double> P;
    plane_line(dl, ml, load_plane<double>(d.pl64 + (int64_t)PL_STRIDE * d.fgrp[FAM][i]), P, false);
    if (!P.degenerate) rel = fmin(rel, image_line_normal(C, P.d2, P.m2));
  }
  return rel;
}

// ---------------------------------------------------------------------------
// linearisation: one lane per record
template <int FAM, typename T, int CD> __global__ __launch_bounds__(256) void k_lin(Dev d) {
  using F = Fam<FAM, CD>;
  using SL = Slot<FAM, CD>;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.fn[FAM]) return;
  const int f = d.ffeat[FAM][i];
  T mT[4] = {0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < F::MEAS; ++k) mT[k] = (T)d.fmeas[FAM][i * F::MEAS + k];
  T v[SL::STRIDE];
#pragma unroll
  for (int k = 0; k < SL::STRIDE; ++k) v[k] = 0;
  T r[F::ROWS];
  T* Jc = v + SL::OC;
  T* Jg = v + SL::OG;
  T* Jf = v + SL::OF;
  const T* camT = (const T*)d.camT;
  const T* ptT = (const T*)d.ptT;
  const T* lnT = (const T*)d.lnT;
  const T* plT = (const T*)d.plT;
  const T* vpT = (const T*)d.vpT;
  if constexpr (FAM == 5) {
    const int g = d.fgrp[FAM][i];
    jac_R5<T>(load_line<T>(lnT + (int64_t)LN_STRIDE * f), load_vp<T>(vpT + (int64_t)VP_STRIDE * g), r, Jg, Jf);
  } else if constexpr (FAM == 8) {
    const T X[3] = {ptT[(int64_t)PT_STRIDE * f], ptT[(int64_t)PT_STRIDE * f + 1], ptT[(int64_t)PT_STRIDE * f + 2]};
    jac_R12<T>(X, load_plane<T>(plT + (int64_t)PL_STRIDE * d.fgrp[FAM][i]), r, Jg, Jf);
  } else {
    const int c = d.fcam[FAM][i];
    Cam<T> C = load_cam<T>(camT + (int64_t)CAM_STRIDE * c);
    if constexpr (FAM == 1 || FAM == 3 || FAM == 6 || FAM == 9) {
      T X[3] = {ptT[(int64_t)PT_STRIDE * f], ptT[(int64_t)PT_STRIDE * f + 1], ptT[(int64_t)PT_STRIDE * f + 2]};
      if constexpr (FAM == 1) jac_R1<T, CD>(C, X, mT, r, Jc, Jf);
      if constexpr (FAM == 3) {
        // a difference of two nearly equal projection Jacobians: evaluated in
        // FP64 from the master parameters, stored in T
        double r3[2], jc3[2 * SL::NC], jg3[6], jf3[6];
        const double* X64 = d.pt64 + (int64_t)PT_STRIDE * f;
        jac_R3<double, CD>(load_cam<double>(d.cam64 + (int64_t)CAM_STRIDE * c), X64,
                           load_plane<double>(d.pl64 + (int64_t)PL_STRIDE * d.fgrp[FAM][i]), r3, jc3, jg3, jf3);
#pragma unroll
        for (int k = 0; k < 2 * SL::NC; ++k) Jc[k] = (T)jc3[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) { Jg[k] = (T)jg3[k]; Jf[k] = (T)jf3[k]; }
      }
      if constexpr (FAM == 6) jac_R6<T, CD>(C, X, mT, r, Jc, Jf);
      if constexpr (FAM == 9) {
        // a difference of two nearly equal projections, like R3: FP64 from the master
        // parameters (the cuboid face chosen in FP64), stored in T
        double r9[2], jc9[2 * SL::NC], jg9[2 * SH_DOF], jf9[6];
        const double* X64 = d.pt64 + (int64_t)PT_STRIDE * f;
        const double* S64 = d.sh64 + (int64_t)SH_STRIDE * d.fgrp[FAM][i];
        jac_R13<double, CD>(load_cam<double>(d.cam64 + (int64_t)CAM_STRIDE * c), X64, S64,
                            shape_type(S64) == SH_CUBOID ? cuboid_face<double>(S64, X64) : 0, r9, jc9, jg9, jf9);
#pragma unroll
        for (int k = 0; k < 2 * SL::NC; ++k) Jc[k] = (T)jc9[k];
#pragma unroll
        for (int k = 0; k < 2 * SH_DOF; ++k) Jg[k] = (T)jg9[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) Jf[k] = (T)jf9[k];
      }
    } else {
      Line<T> L = load_line<T>(lnT + (int64_t)LN_STRIDE * f);
      if constexpr (FAM == 2) jac_R2<T, CD>(C, L, mT, r, Jc, Jf);
      if constexpr (FAM == 4) {
        // difference of two nearly equal line projections: FP64, stored in T
        double m64[4], r4[4], jc4[4 * SL::NC], jg4[12], jf4[16];
#pragma unroll
        for (int k = 0; k < 4; ++k) m64[k] = d.fmeas[FAM][i * 4 + k];
        jac_R4<double, CD>(load_cam<double>(d.cam64 + (int64_t)CAM_STRIDE * c),
                           load_line<double>(d.ln64 + (int64_t)LN_STRIDE * f),
                           load_plane<double>(d.pl64 + (int64_t)PL_STRIDE * d.fgrp[FAM][i]), m64, r4, jc4, jg4, jf4);
#pragma unroll
        for (int k = 0; k < 4 * SL::NC; ++k) Jc[k] = (T)jc4[k];
#pragma unroll
        for (int k = 0; k < 12; ++k) Jg[k] = (T)jg4[k];
#pragma unroll
        for (int k = 0; k < 16; ++k) Jf[k] = (T)jf4[k];
      }
      if constexpr (FAM == 7) jac_R7<T, CD>(C, L, mT, r, Jc, Jf);
      if constexpr (FAM == 10) {
        // like R4: FP64 from the master parameters, the face chosen in FP64, stored in T
        double m64[4], r10[4], jc10[4 * SL::NC], jg10[4 * SH_DOF], jf10[16], dl[3], ml[3];
#pragma unroll
        for (int k = 0; k < 4; ++k) m64[k] = d.fmeas[FAM][i * 4 + k];
        const Line<double> L64 = load_line<double>(d.ln64 + (int64_t)LN_STRIDE * f);
        const double* S64 = d.sh64 + (int64_t)SH_STRIDE * d.fgrp[FAM][i];
        line_dm(L64, dl, ml);
        jac_R14<double, CD>(load_cam<double>(d.cam64 + (int64_t)CAM_STRIDE * c), L64, S64,
                            cuboid_face_line<double>(S64, dl, ml), m64, r10, jc10, jg10, jf10);
#pragma unroll
        for (int k = 0; k < 4 * SL::NC; ++k) Jc[k] = (T)jc10[k];
#pragma unroll
        for (int k = 0; k < 4 * SH_DOF; ++k) Jg[k] = (T)jg10[k];
#pragma unroll
        for (int k = 0; k < 16; ++k) Jf[k] = (T)jf10[k];
      }
    }
  }
  // nearly degenerate image line (relative normal below DEGENERATE_IMAGE_LINE):
  // counted.  The FP64 path keeps the exact Jacobian.  The FP32 path evaluates
  // it in FP64 below FP64_IMAGE_LINE and scales it by rel / DEGENERATE_IMAGE_LINE
  // below the threshold; a Jacobian that is still not finite in T is dropped
  // (the residual stays in the cost either way)
  double jscale = 1.0;
  bool degenerate = false;
  if constexpr (FAM == 2 || FAM == 4 || FAM == 7) {
    const double rel = line_record_normal<FAM>(d, i, f);
    degenerate = rel < DEGENERATE_IMAGE_LINE;
    if constexpr (sizeof(T) < sizeof(double)) {
      if constexpr (FAM == 2 || FAM == 7) {
        if (rel < FP64_IMAGE_LINE) {
          double m64[4] = {0, 0, 0, 0}, r64j[4], jc64[F::ROWS * SL::NC], jf64[F::ROWS * 4];
#pragma unroll
          for (int k = 0; k < F::MEAS; ++k) m64[k] = d.fmeas[FAM][i * F::MEAS + k];
          const Cam<double> C64 = load_cam<double>(d.cam64 + (int64_t)CAM_STRIDE * d.fcam[FAM][i]);
          const Line<double> L64 = load_line<double>(d.ln64 + (int64_t)LN_STRIDE * f);
          if constexpr (FAM == 2) jac_R2<double, CD>(C64, L64, m64, r64j, jc64, jf64);
          else jac_R7<double, CD>(C64, L64, m64, r64j, jc64, jf64);
#pragma unroll
          for (int k = 0; k < F::ROWS * SL::NC; ++k) Jc[k] = (T)jc64[k];
#pragma unroll
          for (int k = 0; k < F::ROWS * 4; ++k) Jf[k] = (T)jf64[k];
        }
      }
      jscale = fmin(1.0, rel / DEGENERATE_IMAGE_LINE);
    }
  }
  bool finite = true;
#pragma unroll
  for (int k = 0; k < SL::USED; ++k) finite = finite && isfinite(v[k]);
  if (!finite) jscale = 0.0;
  if (degenerate || !finite) atomicAdd(&d.scal[SC_NDEG], 1.0);
  // residual in FP64 from the FP64 parameters, robust IRLS scale
  double r64[F::ROWS];
  residual64<FAM>(d, i, d.cam64, d.pt64, d.ln64, d.pl64, d.vp64, d.sh64, r64);
  double s = 0;
#pragma unroll
  for (int k = 0; k < F::ROWS; ++k) s += r64[k] * r64[k];
  double rho, drho;
  loss_eval<double>(d.lkind[FAM], d.lscale[FAM], s, rho, drho);
  const double ws = record_masked<FAM>(d, i, f) ? 0.0 : sqrt(d.lweight[FAM] * drho);
  T* ro = ((T*)d.fres[FAM]) + i * F::ROWS;
#pragma unroll
  for (int k = 0; k < F::ROWS; ++k) ro[k] = (T)(ws * r64[k]);
  if constexpr (FAM <= 4) {
    if (d.cmres[FAM]) {
      T* rc = ((T*)d.cmres[FAM]) + (int64_t)d.cmpos[FAM][i] * F::ROWS;
#pragma unroll
      for (int k = 0; k < F::ROWS; ++k) rc[k] = (T)(ws * r64[k]);
    }
  }
  const T wsT = (T)(ws * jscale);
#pragma unroll
  for (int k = 0; k < SL::USED; ++k) v[k] = jscale > 0.0 ? v[k] * wsT : T(0);
  store_vec(((T*)d.frec[FAM]) + i * SL::STRIDE, v);
  if constexpr (FAM <= 4) {
    if (d.cmrec[FAM]) store_vec(((T*)d.cmrec[FAM]) + (int64_t)d.cmpos[FAM][i] * SL::STRIDE, v);
  }
}

void launch_linearize(const Dev& d, hipStream_t s) {
  BA_DISPATCH_T_CD(d, {
    if (d.fn[1]) k_lin<1, T, CD><<<nblk(d.fn[1], 256), 256, 0, s>>>(d);
    if (d.fn[2]) k_lin<2, T, CD><<<nblk(d.fn[2], 256), 256, 0, s>>>(d);
    if (d.fn[3]) k_lin<3, T, CD><<<nblk(d.fn[3], 256), 256, 0, s>>>(d);
    if (d.fn[4]) k_lin<4, T, CD><<<nblk(d.fn[4], 256), 256, 0, s>>>(d);
    if (d.fn[5]) k_lin<5, T, CD><<<nblk(d.fn[5], 256), 256, 0, s>>>(d);
    if (d.fn[6]) k_lin<6, T, CD><<<nblk(d.fn[6], 256), 256, 0, s>>>(d);
    if (d.fn[7]) k_lin<7, T, CD><<<nblk(d.fn[7], 256), 256, 0, s>>>(d);
    if (d.fn[8]) k_lin<8, T, CD><<<nblk(d.fn[8], 256), 256, 0, s>>>(d);
    if (d.fn[9]) k_lin<9, T, CD><<<nblk(d.fn[9], 256), 256, 0, s>>>(d);
    if (d.fn[10]) k_lin<10, T, CD><<<nblk(d.fn[10], 256), 256, 0, s>>>(d);
  });
  launch_rel_linearize(d, s);
}

// ---------------------------------------------------------------------------
// FP64 cost: one lane per record, per-workgroup partial sums
template <int FAM> __global__ __launch_bounds__(256) void k_cost(Dev d, int candidate, double* part) {
  __shared__ double lds[8];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0;
  if (i < d.fn[FAM] && !record_masked<FAM>(d, i, d.ffeat[FAM][i])) {
    double r[4];
    if (candidate) residual64<FAM>(d, i, d.cam64n, d.pt64n, d.ln64n, d.pl64n, d.vp64n, d.sh64n, r);
    else residual64<FAM>(d, i, d.cam64, d.pt64, d.ln64, d.pl64, d.vp64, d.sh64, r);
    double s = 0;
#pragma unroll
    for (int k = 0; k < Fam<FAM, 9>::ROWS; ++k) s += r[k] * r[k];
    double rho, drho;
    loss_eval<double>(d.lkind[FAM], d.lscale[FAM], s, rho, drho);
    e = 0.5 * d.lweight[FAM] * rho;
  }
  e = wave_sum(e);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[w] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += lds[k];
    part[blockIdx.x] = t;
  }
}

// sum partials [0, n) into scal[SC_E] and, excluding [x0, x1), scal[SC_EPIX]
__global__ __launch_bounds__(1024) void k_cost_final(const double* part, int n, int x0, int x1, double* scal) {
  __shared__ double lds[2 * 17];
  double v[2] = {0, 0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    v[0] += part[i];
    if (i < x0 || i >= x1) v[1] += part[i];
  }
  double* o = block_sum_arr<double, 2>(v, lds);
  if (threadIdx.x == 0) { scal[SC_E] = o[0]; scal[SC_EPIX] = o[1]; }
}

void launch_cost(const Dev& d, bool candidate, hipStream_t s) {
  // the angular terms (VP-line records, then the inter-group relations) and the metric
  // 3D point-to-plane records take one contiguous range [x0, x1) of the partials,
  // which E_pix leaves out
  int off = 0, x0 = -1, x1 = 0;
  auto go = [&](int fam) {
    if (!d.fn[fam]) return;
    unsigned nb = nblk(d.fn[fam], 256);
    if (fam == 5) x0 = off;
    switch (fam) {
      case 1: k_cost<1><<<nb, 256, 0, s>>>(d, candidate, d.red + off); break;
      case 2: k_cost<2><<<nb, 256, 0, s>>>(d, candidate, d.red + off); break;
      case 3: k_cost<3><<<nb, 256, 0, s>>>(d, candidate, d.red + off); break;
      case 4: k_cost<4><<<nb, 256, 0, s>>>(d, candidate, d.red + off); break;
      case 5: k_cost<5><<<nb, 256, 0, s>>>(d, candidate, d.red + off); break;
      case 6: k_cost<6><<<nb, 256, 0, s>>>(d, candidate, d.red + off); break;
      case 7: k_cost<7><<<nb, 256, 0, s>>>(d, candidate, d.red + off); break;
      case 8: k_cost<8><<<nb, 256, 0, s>>>(d, candidate, d.red + off); break;
      case 9: k_cost<9><<<nb, 256, 0, s>>>(d, candidate, d.red + off); break;
      case 10: k_cost<10><<<nb, 256, 0, s>>>(d, candidate, d.red + off); break;
    }
    off += (int)nb;
    if (fam == 5) x1 = off;
  };
  for (int fam = 1; fam <= 5; ++fam) go(fam);
  if (d.n_rel) {
    if (x0 < 0) x0 = off;
    launch_rel_cost(d, candidate, d.red + off, s);
    x1 = ++off;
  }
  // the 3D point-to-plane distances are metric, not pixels: in the same range
  if (d.fn[8]) {
    if (x0 < 0) x0 = off;
    go(8);
    x1 = off;
  }
  for (int fam = 6; fam <= 7; ++fam) go(fam);
  for (int fam = 9; fam <= 10; ++fam) go(fam);  // surface groups: pixels
  if (x0 < 0) x0 = x1 = 0;
  k_cost_final<<<1, 1024, 0, s>>>(d.red, off, x0, x1, d.scal);
}

// ---------------------------------------------------------------------------
// feature blocks
template <int FAM, typename T, int CD, int NF, typename A>
__device__ __forceinline__ void acc_feature(const Dev& d, int f, A (&V)[NF * (NF + 1) / 2], A (&g)[NF]) {
  using SL = Slot<FAM, CD>;
  if (!d.fn[FAM]) return;
  const int64_t b = d.foff[FAM][f], e = d.foff[FAM][f + 1];
  const T* rec = (const T*)d.frec[FAM];
  const T* res = (const T*)d.fres[FAM];
  for (int64_t i = b; i < e; ++i) {
    T v[SL::STRIDE];
    load_vec(rec + i * SL::STRIDE, v);
#pragma unroll
    for (int row = 0; row < SL::ROWS; ++row) {
      const T* jf = v + SL::OF + row * NF;
      const A rr = (A)res[i * SL::ROWS + row];
#pragma unroll
      for (int a = 0; a < NF; ++a) {
        g[a] += (A)jf[a] * rr;
#pragma unroll
        for (int b2 = a; b2 < NF; ++b2) V[sym<NF>(a, b2)] += (A)jf[a] * (A)jf[b2];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Records of the surface-group families (9, 10: SH_DOF group columns, the largest
// slots) are read one row at a time wherever they are handled, so that they do not
// raise the register budget of the kernels shared with the other families.
template <int FAM, typename T, int CD, int NF, typename A>
__device__ __forceinline__ void acc_feature_rows(const Dev& d, int f, A (&V)[NF * (NF + 1) / 2], A (&g)[NF]) {
  using SL = Slot<FAM, CD>;
  if (!d.fn[FAM]) return;
  const T* rec = (const T*)d.frec[FAM];
  const T* res = (const T*)d.fres[FAM];
  for (int64_t i = d.foff[FAM][f]; i < d.foff[FAM][f + 1]; ++i) {
#pragma unroll 1
    for (int row = 0; row < SL::ROWS; ++row) {
      const T* jf = rec + i * SL::STRIDE + SL::OF + row * NF;
      const A rr = (A)res[i * SL::ROWS + row];
      A j[NF];
#pragma unroll
      for (int a = 0; a < NF; ++a) j[a] = (A)jf[a];
#pragma unroll
      for (int a = 0; a < NF; ++a) {
        g[a] += j[a] * rr;
#pragma unroll
        for (int b2 = a; b2 < NF; ++b2) V[sym<NF>(a, b2)] += j[a] * j[b2];
      }
    }
  }
}

// U_cc, g_c of one surface-group record
template <int FAM, typename T, int CD>
__device__ __forceinline__ void cam_a_rows(const Dev& d, int64_t i, T (&U)[CD * (CD + 1) / 2], T (&g)[CD]) {
  using SL = Slot<FAM, CD>;
  const T* sl = (const T*)d.frec[FAM] + i * SL::STRIDE;
  const T* res = (const T*)d.fres[FAM] + i * SL::ROWS;
#pragma unroll 1
  for (int row = 0; row < SL::ROWS; ++row) {
    T jc[SL::NC];
#pragma unroll
    for (int k = 0; k < SL::NC; ++k) jc[k] = sl[SL::OC + row * SL::NC + k];
    const T rr = res[row];
#pragma unroll
    for (int a = 0; a < SL::NC; ++a) {
      g[a] += jc[a] * rr;
#pragma unroll
      for (int b = a; b < SL::NC; ++b) U[sym<CD>(a, b)] += jc[a] * jc[b];
    }
  }
}

// W += J_o^T J_f of one surface-group record, o the camera (OUT 0) or shape (OUT 1) columns
template <int FAM, int OUT, typename T, int CD, int N, int NF>
__device__ __forceinline__ void addW_rows(const Dev& d, int64_t i, T (&W)[N][NF]) {
  using SL = Slot<FAM, CD>;
  constexpr int NK = OUT == 0 ? SL::NC : SL::NG, O = OUT == 0 ? SL::OC : SL::OG;
  static_assert(N >= NK, "output rows");
  const T* sl = (const T*)d.frec[FAM] + i * SL::STRIDE;
#pragma unroll 1
  for (int row = 0; row < SL::ROWS; ++row) {
    T jo[NK], jf[NF];
#pragma unroll
    for (int k = 0; k < NK; ++k) jo[k] = sl[O + row * NK + k];
#pragma unroll
    for (int k = 0; k < NF; ++k) jf[k] = sl[SL::OF + row * NF + k];
#pragma unroll
    for (int a = 0; a < NK; ++a)
#pragma unroll
      for (int b = 0; b < NF; ++b) W[a][b] += jo[a] * jf[b];
  }
}





// S Z sweeps, output rows, with the Z rows of the output side in registers: zk holds the
// rows of the record's camera (OUT 0, a camera's sweep) or of its shape (OUT 1, a shape's
// chunk), which the caller keeps for all its records; the other side's rows and s_f are
// read from the panel. The loads of a row are independent of one another, so their
// latencies overlap; the rows go one at a time to bound the registers.
template <int FAM, int OUT, typename T, int CD, int CPL, int NK>
__device__ __forceinline__ void sz_shape_rec(const Dev& d, int64_t i, const T (&zk)[NK][CPL], const T* zr, const T* s,
                                             double (&acc)[NK][CPL]) {
  using SL = Slot<FAM, CD>;
  using F = Fam<FAM, CD>;
  constexpr int NU = OUT == 0 ? SL::NC : SL::NG, NO = OUT == 0 ? SL::NG : SL::NC;
  static_assert(NK >= NU, "the output side's rows (a line's camera columns are the first NC)");
  constexpr int OK = OUT == 0 ? SL::OC : SL::OG, OO = OUT == 0 ? SL::OG : SL::OC;
  const T* sl = (const T*)d.frec[FAM] + i * SL::STRIDE;
  const int64_t e = OUT == 0 ? (int64_t)a_grp(d, F::GT, d.fgrp[FAM][i]) : (int64_t)CD * d.fcam[FAM][i];
  T zo[NO][CPL], sf[SL::NF][CPL];
#pragma unroll
  for (int k = 0; k < NO; ++k)
#pragma unroll
    for (int c = 0; c < CPL; ++c) zo[k][c] = zr[(e + k) * SZ_COLS + c];
#pragma unroll
  for (int a = 0; a < SL::NF; ++a)
#pragma unroll
    for (int c = 0; c < CPL; ++c) sf[a][c] = s[a * SZ_COLS + c];
#pragma unroll 1
  for (int row = 0; row < SL::ROWS; ++row) {
    T jk[NU], u[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) u[c] = 0;
#pragma unroll
    for (int k = 0; k < NU; ++k) {
      jk[k] = sl[OK + row * NU + k];
#pragma unroll
      for (int c = 0; c < CPL; ++c) u[c] += jk[k] * zk[k][c];
    }
#pragma unroll
    for (int k = 0; k < NO; ++k) {
      const T j = sl[OO + row * NO + k];
#pragma unroll
      for (int c = 0; c < CPL; ++c) u[c] += j * zo[k][c];
    }
#pragma unroll
    for (int a = 0; a < SL::NF; ++a) {
      const T j = sl[SL::OF + row * SL::NF + a];
#pragma unroll
      for (int c = 0; c < CPL; ++c) u[c] -= j * sf[a][c];
    }
#pragma unroll
    for (int k = 0; k < NU; ++k)
#pragma unroll
      for (int c = 0; c < CPL; ++c) acc[k][c] += (double)(jk[k] * u[c]);
  }
}

template <typename T, int CD, int NF, typename A> __device__ __forceinline__ void acc_feature_all(const Dev& d, int f, A (&V)[NF * (NF + 1) / 2], A (&g)[NF]) {
  if constexpr (NF == 3) {
    acc_feature<1, T, CD, 3>(d, f, V, g);
    acc_feature<3, T, CD, 3>(d, f, V, g);
    acc_feature<6, T, CD, 3>(d, f, V, g);
    acc_feature<8, T, CD, 3>(d, f, V, g);
    acc_feature_rows<9, T, CD, 3>(d, f, V, g);
  } else {
    acc_feature<2, T, CD, 4>(d, f, V, g);
    acc_feature<4, T, CD, 4>(d, f, V, g);
    acc_feature<5, T, CD, 4>(d, f, V, g);
    acc_feature<7, T, CD, 4>(d, f, V, g);
    acc_feature_rows<10, T, CD, 4>(d, f, V, g);
  }
}

template <typename T, int CD, int NF> __device__ __forceinline__ void feature_accum_one(const Dev& d, int f) {
  constexpr int NS = NF * (NF + 1) / 2;
  T V[NS], g[NF];
#pragma unroll
  for (int k = 0; k < NS; ++k) V[k] = 0;
#pragma unroll
  for (int k = 0; k < NF; ++k) g[k] = 0;
  acc_feature_all<T, CD, NF, T>(d, f, V, g);
  T* Vo = (T*)(NF == 3 ? d.Vp : d.Vl) + (int64_t)NS * f;
  T* go = (T*)(NF == 3 ? d.gp : d.gl) + (int64_t)NF * f;
  double* Do = (NF == 3 ? d.Dp : d.Dl) + (int64_t)NF * f;
#pragma unroll
  for (int k = 0; k < NS; ++k) Vo[k] = V[k];
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    go[k] = g[k];
    Do[k] = fmin(fmax((double)V[sym<NF>(k, k)], 1e-6), 1e32);
  }
}

template <typename T, int CD> __global__ __launch_bounds__(256) void k_feat_accum(Dev d, int ptiles) {
  if ((int)blockIdx.x < ptiles) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < d.np) feature_accum_one<T, CD, 3>(d, f);
  } else {
    const int f = (blockIdx.x - ptiles) * blockDim.x + threadIdx.x;
    if (f < d.nl) feature_accum_one<T, CD, 4>(d, f);
  }
}

void launch_feature_accum(const Dev& d, hipStream_t s) {
  const int pt = (int)nblk(d.np, 256), lt = (int)nblk(d.nl, 256);
  if (pt + lt == 0) return;
  BA_DISPATCH_T_CD(d, k_feat_accum<T, CD><<<pt + lt, 256, 0, s>>>(d, pt));
}

// |g|_inf over the whole parameter vector: g_a (FP64), then g_f of points and lines (T).
// Non-negative doubles order as their bit patterns, and a NaN's pattern is above every
// finite one and infinity, so a maximum over the patterns also carries a NaN through.
template <typename T> __global__ void k_grad_inf(Dev d) {
  const int64_t na = d.nA, np = 3 * (int64_t)d.np, n = na + np + 4 * (int64_t)d.nl;
  unsigned long long m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = i < na ? d.gA[i] : i < na + np ? (double)((const T*)d.gp)[i - na] : (double)((const T*)d.gl)[i - na - np];
    const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(v));
    m = b > m ? b : m;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long u = __shfl_xor(m, o);
    m = u > m ? u : m;
  }
  if ((threadIdx.x & 63) == 0 && m) atomicMax((unsigned long long*)(d.scal + SC_GINF), m);
}

void launch_grad_inf(const Dev& d, hipStream_t s) {
  launch_zero(d.scal + SC_GINF, sizeof(double), s);
  const int64_t n = d.nA + 3 * (int64_t)d.np + 4 * (int64_t)d.nl;
  if (!n) return;
  const unsigned nb = std::min<unsigned>(nblk(n, 256), 1024);
  if (d.fp64) k_grad_inf<double><<<nb, 256, 0, s>>>(d);
  else k_grad_inf<float><<<nb, 256, 0, s>>>(d);
}

// damped inverse of one feature block; FP32 blocks whose Cholesky fails or
// whose estimated condition exceeds kappa_max are redone in FP64 from the
// stored Jacobians
template <typename T, int CD, int NF> __device__ __forceinline__ int feature_invert_one(const Dev& d, int f, double lam, double kmax) {
  constexpr int NS = NF * (NF + 1) / 2;
  const T* Vin = (const T*)(NF == 3 ? d.Vp : d.Vl) + (int64_t)NS * f;
  const T* gin = (const T*)(NF == 3 ? d.gp : d.gl) + (int64_t)NF * f;
  const double* D = (NF == 3 ? d.Dp : d.Dl) + (int64_t)NF * f;
  T* Vio = (T*)(NF == 3 ? d.Vip : d.Vil) + (int64_t)NS * f;
  T* so = (T*)(NF == 3 ? d.sp : d.sl) + (int64_t)NF * f;
  double* Vio64 = (NF == 3 ? d.Vip64 : d.Vil64) + (int64_t)NS * f;
  uint8_t* flag = (NF == 3 ? d.flp : d.fll) + f;
  T A[NF][NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) {
#pragma unroll
    for (int j = 0; j < NF; ++j) A[i][j] = Vin[sym<NF>(i, j)];
    A[i][i] += (T)(lam * D[i]);
  }
  bool ok = chol<T, NF>(A);
  if (ok) {
    T mx = A[0][0], mn = A[0][0];
#pragma unroll
    for (int i = 1; i < NF; ++i) { mx = fmax(mx, A[i][i]); mn = fmin(mn, A[i][i]); }
    const double kap = ((double)mx / (double)mn) * ((double)mx / (double)mn);
    if (sizeof(T) == 4 && kap > kmax) ok = false;
  }
  if (ok) {
    T Ai[NF][NF];
    chol_inverse<T, NF>(A, Ai);
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      T t = 0;
#pragma unroll
      for (int j = 0; j < NF; ++j) t += Ai[i][j] * gin[j];
      so[i] = t;
#pragma unroll
      for (int j = i; j < NF; ++j) Vio[sym<NF>(i, j)] = Ai[i][j];
    }
    *flag = 0;
    return 0;
  }
  // FP64 path: re-accumulate from the stored Jacobians in double
  double V64[NS], g64[NF];
#pragma unroll
  for (int k = 0; k < NS; ++k) V64[k] = 0;
#pragma unroll
  for (int k = 0; k < NF; ++k) g64[k] = 0;
  acc_feature_all<T, CD, NF, double>(d, f, V64, g64);
  double B[NF][NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) {
#pragma unroll
    for (int j = 0; j < NF; ++j) B[i][j] = V64[sym<NF>(i, j)];
    B[i][i] += lam * D[i];
  }
  double Bi[NF][NF];
  const bool ok64 = chol<double, NF>(B);
  if (ok64) chol_inverse<double, NF>(B, Bi);
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    double t = 0;
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      if (!ok64) Bi[i][j] = 0;
      t += Bi[i][j] * g64[j];
    }
    so[i] = (T)t;
#pragma unroll
    for (int j = i; j < NF; ++j) { Vio64[sym<NF>(i, j)] = Bi[i][j]; Vio[sym<NF>(i, j)] = (T)Bi[i][j]; }
  }
  *flag = ok64 ? 1 : 2;
  return ok64 ? 1 : 2;
}

template <typename T, int CD> __global__ __launch_bounds__(256) void k_feat_inv(Dev d, int ptiles, double lam, double kmax) {
  __shared__ double lds[8];
  int nf = 0;
  if ((int)blockIdx.x < ptiles) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < d.np) nf = feature_invert_one<T, CD, 3>(d, f, lam, kmax);
  } else {
    const int f = (blockIdx.x - ptiles) * blockDim.x + threadIdx.x;
    if (f < d.nl) nf = feature_invert_one<T, CD, 4>(d, f, lam, kmax);
  }
  // FP64 re-inversions (flag 1 or 2) and, of those, failed FP64 Cholesky (flag 2)
  const double c = wave_sum((double)(nf != 0)), c2 = wave_sum((double)(nf == 2));
  if ((threadIdx.x & 63) == 0) {
    lds[threadIdx.x >> 6] = c;
    lds[4 + (threadIdx.x >> 6)] = c2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0, t2 = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { t += lds[k]; t2 += lds[4 + k]; }
    if (t > 0) atomicAdd(&d.scal[SC_NFLAG], t);
    if (t2 > 0) atomicAdd(&d.scal[SC_NFAIL], t2);
  }
}

void launch_feature_invert(const Dev& d, double lambda, double kappa_max, hipStream_t s) {
  const int pt = (int)nblk(d.np, 256), lt = (int)nblk(d.nl, 256);
  if (pt + lt == 0) return;
  BA_DISPATCH_T_CD(d, k_feat_inv<T, CD><<<pt + lt, 256, 0, s>>>(d, pt, lambda, kappa_max));
}

// apply a feature inverse (packed, or FP64 for flagged features)
template <typename T, int NF> __device__ __forceinline__ void apply_vinv(const Dev& d, int f, const T (&q)[NF], T (&s)[NF]) {
  constexpr int NS = NF * (NF + 1) / 2;
  const uint8_t fl = (NF == 3 ? d.flp : d.fll)[f];
  if (fl) {
    const double* M = (NF == 3 ? d.Vip64 : d.Vil64) + (int64_t)NS * f;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      double t = 0;
#pragma unroll
      for (int j = 0; j < NF; ++j) t += M[sym<NF>(i, j)] * (double)q[j];
      s[i] = (T)t;
    }
  } else {
    const T* M = (const T*)(NF == 3 ? d.Vip : d.Vil) + (int64_t)NS * f;
    T m[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) m[k] = M[k];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      T t = 0;
#pragma unroll
      for (int j = 0; j < NF; ++j) t += m[sym<NF>(i, j)] * q[j];
      s[i] = t;
    }
  }
}

template <typename T, int NF> __device__ __forceinline__ void load_vinv_full(const Dev& d, int f, T (&M)[NF][NF]) {
  constexpr int NS = NF * (NF + 1) / 2;
  const uint8_t fl = (NF == 3 ? d.flp : d.fll)[f];
  if (fl) {
    const double* P = (NF == 3 ? d.Vip64 : d.Vil64) + (int64_t)NS * f;
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) M[i][j] = (T)P[sym<NF>(i, j)];
  } else {
    const T* P = (const T*)(NF == 3 ? d.Vip : d.Vil) + (int64_t)NS * f;
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) M[i][j] = P[sym<NF>(i, j)];
  }
}

// ---------------------------------------------------------------------------
// camera pass A: U_cc, g_c (one workgroup per camera)
template <int FAM, typename T, int CD>
__device__ __forceinline__ void cam_a_slot(const T* slot, const T* res, T (&U)[CD * (CD + 1) / 2], T (&g)[CD]) {
  using SL = Slot<FAM, CD>;
  T v[SL::STRIDE];
  load_vec(slot, v);
#pragma unroll
  for (int row = 0; row < SL::ROWS; ++row) {
    const T* jc = v + SL::OC + row * SL::NC;
    const T rr = res[row];
#pragma unroll
    for (int a = 0; a < SL::NC; ++a) {
      g[a] += jc[a] * rr;
#pragma unroll
      for (int b = a; b < SL::NC; ++b) U[sym<CD>(a, b)] += jc[a] * jc[b];
    }
  }
}

template <int FAM, typename T, int CD> __device__ __forceinline__ void cam_a_rec(const Dev& d, int64_t i, T (&U)[CD * (CD + 1) / 2], T (&g)[CD]) {
  using SL = Slot<FAM, CD>;
  T v[SL::STRIDE];
  load_vec(((const T*)d.frec[FAM]) + i * SL::STRIDE, v);
  const T* res = ((const T*)d.fres[FAM]) + i * SL::ROWS;
#pragma unroll
  for (int row = 0; row < SL::ROWS; ++row) {
    const T* jc = v + SL::OC + row * SL::NC;
    const T rr = res[row];
#pragma unroll
    for (int a = 0; a < SL::NC; ++a) {
      g[a] += jc[a] * rr;
#pragma unroll
      for (int b = a; b < SL::NC; ++b) U[sym<CD>(a, b)] += jc[a] * jc[b];
    }
  }
}

template <typename T, int CD> __global__ __launch_bounds__(256) void k_cam_a(Dev d) {
  constexpr int NS = CD * (CD + 1) / 2;
  constexpr int K = NS + CD;
  __shared__ T lds[(4 + 1) * K];
  const int c = d.cam_order[blockIdx.x];
  T acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0;
  T(&U)[NS] = *reinterpret_cast<T(*)[NS]>(acc);
  T(&g)[CD] = *reinterpret_cast<T(*)[CD]>(acc + NS);
  if (d.fn[1]) {
    // observation slots and their aligned plane slots from the camera-major copies
    for (int j = d.po_off[c] + threadIdx.x; j < d.po_off[c + 1]; j += blockDim.x) {
      cam_a_slot<1, T, CD>((const T*)d.cmrec[1] + (int64_t)j * Slot<1, CD>::STRIDE, (const T*)d.cmres[1] + (int64_t)j * Slot<1, CD>::ROWS, U, g);
      const int k = d.cmal[1][j];
      if (k >= 0)
        cam_a_slot<3, T, CD>((const T*)d.cmrec[3] + (int64_t)k * Slot<3, CD>::STRIDE, (const T*)d.cmres[3] + (int64_t)k * Slot<3, CD>::ROWS, U, g);
    }
  }
  // the camera's point-on-shape and line-on-cuboid records, in loops of their own (inside
  // the observation loops every wavefront would take both paths)
  if (d.shc_off[0])
    for (int j = d.shc_off[0][c] + threadIdx.x; j < d.shc_off[0][c + 1]; j += blockDim.x) cam_a_rows<9, T, CD>(d, d.shc_rec[0][j], U, g);
  if (d.shc_off[1])
    for (int j = d.shc_off[1][c] + threadIdx.x; j < d.shc_off[1][c + 1]; j += blockDim.x) cam_a_rows<10, T, CD>(d, d.shc_rec[1][j], U, g);
  if (d.fn[6]) {
    for (int j = d.px_off[c] + threadIdx.x; j < d.px_off[c + 1]; j += blockDim.x)
      for (int64_t i = d.px_start[j]; i < d.px_start[j] + d.px_cnt[j]; ++i) cam_a_rec<6, T, CD>(d, i, U, g);
  }
  if (d.fn[2]) {
    for (int j = d.lo_off[c] + threadIdx.x; j < d.lo_off[c + 1]; j += blockDim.x) {
      cam_a_slot<2, T, CD>((const T*)d.cmrec[2] + (int64_t)j * Slot<2, CD>::STRIDE, (const T*)d.cmres[2] + (int64_t)j * Slot<2, CD>::ROWS, U, g);
      const int k = d.cmal[2][j];
      if (k >= 0)
        cam_a_slot<4, T, CD>((const T*)d.cmrec[4] + (int64_t)k * Slot<4, CD>::STRIDE, (const T*)d.cmres[4] + (int64_t)k * Slot<4, CD>::ROWS, U, g);
    }
  }
  if (d.fn[7]) {
    for (int j = d.lx_off[c] + threadIdx.x; j < d.lx_off[c + 1]; j += blockDim.x)
      for (int64_t i = d.lx_start[j]; i < d.lx_start[j] + d.lx_cnt[j]; ++i) cam_a_rec<7, T, CD>(d, i, U, g);
  }
  T* o = block_sum_arr<T, K>(acc, lds);
  for (int k = threadIdx.x; k < CD * CD; k += blockDim.x) {
    const int a = k / CD, b = k % CD;
    d.Ucam[(int64_t)c * CD * CD + k] = (double)o[sym<CD>(a, b)];
  }
  for (int k = threadIdx.x; k < CD; k += blockDim.x) {
    d.gA[CD * c + k] = (double)o[NS + k];
    d.DA[CD * c + k] = fmin(fmax((double)o[sym<CD>(k, k)], 1e-6), 1e32);
  }
}

// group pass A: one workgroup per plane, then per VP
template <int FAM, typename T, int CD, int NG> __device__ __forceinline__ void grp_a_rec(const Dev& d, int64_t i, T* U, T* g) {
  using SL = Slot<FAM, CD>;
  T v[SL::STRIDE];
  load_vec(((const T*)d.frec[FAM]) + i * SL::STRIDE, v);
  const T* res = ((const T*)d.fres[FAM]) + i * SL::ROWS;
#pragma unroll
  for (int row = 0; row < SL::ROWS; ++row) {
    const T* jg = v + SL::OG + row * NG;
    const T rr = res[row];
#pragma unroll
    for (int a = 0; a < NG; ++a) {
      g[a] += jg[a] * rr;
#pragma unroll
      for (int b = a; b < NG; ++b) U[sym<NG>(a, b)] += jg[a] * jg[b];
    }
  }
}

template <typename T, int CD> __global__ __launch_bounds__(256) void k_grp_a(Dev d) {
  __shared__ T lds[5 * 9];
  if ((int)blockIdx.x < d.ng) {
    const int g = blockIdx.x;
    T acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0;
    // points of the plane: its plane-association records (R3) and 3D point-to-plane
    // records (family 8); a point's records of either family may name other planes
    if (d.fn[3] || d.fn[8])
      for (int j = d.plp_off[g] + threadIdx.x; j < d.plp_off[g + 1]; j += blockDim.x) {
        const int f = d.plp[j];
        for (int64_t i = d.foff[3][f]; i < d.foff[3][f + 1]; ++i)
          if (d.fgrp[3][i] == g) grp_a_rec<3, T, CD, 3>(d, i, acc, acc + 6);
        for (int64_t i = d.foff[8][f]; i < d.foff[8][f + 1]; ++i)
          if (d.fgrp[8][i] == g) grp_a_rec<8, T, CD, 3>(d, i, acc, acc + 6);
      }
    if (d.fn[4])
      for (int j = d.pll_off[g] + threadIdx.x; j < d.pll_off[g + 1]; j += blockDim.x) {
        const int f = d.pll[j];
        for (int64_t i = d.foff[4][f]; i < d.foff[4][f + 1]; ++i) grp_a_rec<4, T, CD, 3>(d, i, acc, acc + 6);
      }
    T* o = block_sum_arr<T, 9>(acc, lds);
    if (threadIdx.x < 9) {
      const int a = threadIdx.x / 3, b = threadIdx.x % 3;
      d.Upl[9 * g + threadIdx.x] = (double)o[sym<3>(a, b)];
    }
    if (threadIdx.x < 3) {
      const int k = threadIdx.x;
      d.gA[d.offPl + 3 * g + k] = (double)o[6 + k];
      d.DA[d.offPl + 3 * g + k] = fmin(fmax((double)o[sym<3>(k, k)], 1e-6), 1e32);
    }
  } else {
    const int v = blockIdx.x - d.ng;
    T acc[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) acc[k] = 0;
    for (int j = d.vpm_off[v] + threadIdx.x; j < d.vpm_off[v + 1]; j += blockDim.x)
      grp_a_rec<5, T, CD, 2>(d, d.vpm[j], acc, acc + 3);
    T* o = block_sum_arr<T, 5>(acc, lds);
    if (threadIdx.x < 4) {
      const int a = threadIdx.x / 2, b = threadIdx.x % 2;
      d.Uvp[4 * v + threadIdx.x] = (double)o[sym<2>(a, b)];
    }
    if (threadIdx.x < 2) {
      const int k = threadIdx.x;
      d.gA[d.offVp + 2 * v + k] = (double)o[3 + k];
      d.DA[d.offVp + 2 * v + k] = fmin(fmax((double)o[sym<2>(k, k)], 1e-6), 1e32);
    }
  }
}

void launch_camera_pass_a(const Dev& d, hipStream_t s) {
  BA_DISPATCH_T_CD(d, {
    if (d.nc) k_cam_a<T, CD><<<d.nc, 256, 0, s>>>(d);
    if (d.ng + d.nv) k_grp_a<T, CD><<<d.ng + d.nv, 256, 0, s>>>(d);
  });
  launch_shape_pass_a(d, s);
  launch_rel_a(d, s);
}

// ---------------------------------------------------------------------------
// camera pass B: damped diagonal blocks of S and b with pair-summed W_af
template <int FAM, typename T, int CD, int NF> __device__ __forceinline__ void addW_slot(const T* slot, T (&W)[CD][NF]) {
  using SL = Slot<FAM, CD>;
  T v[SL::STRIDE];
  load_vec(slot, v);
#pragma unroll
  for (int row = 0; row < SL::ROWS; ++row) {
    const T* jc = v + SL::OC + row * SL::NC;
    const T* jf = v + SL::OF + row * NF;
#pragma unroll
    for (int a = 0; a < SL::NC; ++a)
#pragma unroll
      for (int b = 0; b < NF; ++b) W[a][b] += jc[a] * jf[b];
  }
}

template <int FAM, typename T, int CD, int NF> __device__ __forceinline__ void addW_cam(const Dev& d, int64_t i, T (&W)[CD][NF]) {
  using SL = Slot<FAM, CD>;
  T v[SL::STRIDE];
  load_vec(((const T*)d.frec[FAM]) + i * SL::STRIDE, v);
#pragma unroll
  for (int row = 0; row < SL::ROWS; ++row) {
    const T* jc = v + SL::OC + row * SL::NC;
    const T* jf = v + SL::OF + row * NF;
#pragma unroll
    for (int a = 0; a < SL::NC; ++a)
#pragma unroll
      for (int b = 0; b < NF; ++b) W[a][b] += jc[a] * jf[b];
  }
}

// C -= W V^-1 W^T ; bb += W s   for the pair's feature f
template <typename T, int N, int NF> __device__ __forceinline__ void pair_contrib(const Dev& d, int f, const T (&W)[N][NF],
                                                                               T* C, T* bb) {
  T M[NF][NF];
  load_vinv_full<T, NF>(d, f, M);
  const T* sv = (const T*)(NF == 3 ? d.sp : d.sl) + (int64_t)NF * f;
  T s[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) s[k] = sv[k];
  T Y[N][NF];
#pragma unroll
  for (int a = 0; a < N; ++a) {
#pragma unroll
    for (int b = 0; b < NF; ++b) {
      T t = 0;
#pragma unroll
      for (int k = 0; k < NF; ++k) t += W[a][k] * M[k][b];
      Y[a][b] = t;
    }
    T t = 0;
#pragma unroll
    for (int k = 0; k < NF; ++k) t += W[a][k] * s[k];
    bb[a] += t;
  }
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = a; b < N; ++b) {
      T t = 0;
#pragma unroll
      for (int k = 0; k < NF; ++k) t += Y[a][k] * W[b][k];
      C[sym<N>(a, b)] -= t;
    }
}

template <typename T, int CD> __global__ __launch_bounds__(256) void k_cam_b(Dev d, double lam) {
  constexpr int NS = CD * (CD + 1) / 2;
  constexpr int K = NS + CD;
  __shared__ T lds[(4 + 1) * K];
  const int c = d.cam_order[blockIdx.x];
  T acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0;
  T* C = acc;
  T* bb = acc + NS;
  if (d.fn[1]) {
    // observation slot and its aligned plane slot from the camera-major copies
    for (int j = d.po_off[c] + threadIdx.x; j < d.po_off[c + 1]; j += blockDim.x) {
      T W[CD][3];
#pragma unroll
      for (int a = 0; a < CD; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) W[a][b] = 0;
      addW_slot<1, T, CD, 3>((const T*)d.cmrec[1] + (int64_t)j * Slot<1, CD>::STRIDE, W);
      const int k = d.cmal[1][j];
      if (k >= 0) addW_slot<3, T, CD, 3>((const T*)d.cmrec[3] + (int64_t)k * Slot<3, CD>::STRIDE, W);
      if (d.shal_p) {
        const int k9 = d.shal_p[j];
        if (k9 >= 0) addW_rows<9, 0, T, CD, CD, 3>(d, k9, W);
      }
      pair_contrib<T, CD, 3>(d, d.cmfeat[1][j], W, C, bb);
    }
  }
  if (d.fn[6]) {
    for (int j = d.px_off[c] + threadIdx.x; j < d.px_off[c + 1]; j += blockDim.x) {
      T W[CD][3];
#pragma unroll
      for (int a = 0; a < CD; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) W[a][b] = 0;
      const int64_t i0 = d.px_start[j];
      for (int64_t i = i0; i < i0 + d.px_cnt[j]; ++i) addW_cam<6, T, CD, 3>(d, i, W);
      pair_contrib<T, CD, 3>(d, d.ffeat[6][i0], W, C, bb);
    }
  }
  if (d.fn[2]) {
    for (int j = d.lo_off[c] + threadIdx.x; j < d.lo_off[c + 1]; j += blockDim.x) {
      T W[CD][4];
#pragma unroll
      for (int a = 0; a < CD; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) W[a][b] = 0;
      addW_slot<2, T, CD, 4>((const T*)d.cmrec[2] + (int64_t)j * Slot<2, CD>::STRIDE, W);
      const int k = d.cmal[2][j];
      if (k >= 0) addW_slot<4, T, CD, 4>((const T*)d.cmrec[4] + (int64_t)k * Slot<4, CD>::STRIDE, W);
      if (d.shal_l) {
        const int k10 = d.shal_l[j];
        if (k10 >= 0) addW_rows<10, 0, T, CD, CD, 4>(d, k10, W);
      }
      pair_contrib<T, CD, 4>(d, d.cmfeat[2][j], W, C, bb);
    }
  }
  if (d.fn[7]) {
    for (int j = d.lx_off[c] + threadIdx.x; j < d.lx_off[c + 1]; j += blockDim.x) {
      T W[CD][4];
#pragma unroll
      for (int a = 0; a < CD; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) W[a][b] = 0;
      const int64_t i0 = d.lx_start[j];
      for (int64_t i = i0; i < i0 + d.lx_cnt[j]; ++i) addW_cam<7, T, CD, 4>(d, i, W);
      pair_contrib<T, CD, 4>(d, d.ffeat[7][i0], W, C, bb);
    }
  }
  T* o = block_sum_arr<T, K>(acc, lds);
  for (int k = threadIdx.x; k < CD * CD; k += blockDim.x) {
    const int a = k / CD, b = k % CD;
    const int64_t idx = (int64_t)c * CD * CD + k;
    double v = d.Ucam[idx] + (double)o[sym<CD>(a, b)];
    if (a == b) v += lam * d.DA[CD * c + a];
    d.Scam[idx] = v;
  }
  for (int k = threadIdx.x; k < CD; k += blockDim.x) d.bA[CD * c + k] = -d.gA[CD * c + k] + (double)o[NS + k];
}

template <int FAM, typename T, int CD, int NG, int NF> __device__ __forceinline__ void addW_grp(const Dev& d, int64_t i, T (&W)[NG][NF]) {
  using SL = Slot<FAM, CD>;
  T v[SL::STRIDE];
  load_vec(((const T*)d.frec[FAM]) + i * SL::STRIDE, v);
#pragma unroll
  for (int row = 0; row < SL::ROWS; ++row) {
    const T* jg = v + SL::OG + row * NG;
    const T* jf = v + SL::OF + row * NF;
#pragma unroll
    for (int a = 0; a < NG; ++a)
#pragma unroll
      for (int b = 0; b < NF; ++b) W[a][b] += jg[a] * jf[b];
  }
}

template <typename T, int CD> __global__ __launch_bounds__(256) void k_grp_b(Dev d, double lam) {
  __shared__ T lds[5 * 9];
  if ((int)blockIdx.x < d.ng) {
    const int g = blockIdx.x;
    T acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0;
    if (d.fn[3] || d.fn[8])
      for (int j = d.plp_off[g] + threadIdx.x; j < d.plp_off[g + 1]; j += blockDim.x) {
        const int f = d.plp[j];
        T W[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int64_t i = d.foff[3][f]; i < d.foff[3][f + 1]; ++i)
          if (d.fgrp[3][i] == g) addW_grp<3, T, CD, 3, 3>(d, i, W);
        for (int64_t i = d.foff[8][f]; i < d.foff[8][f + 1]; ++i)
          if (d.fgrp[8][i] == g) addW_grp<8, T, CD, 3, 3>(d, i, W);
        pair_contrib<T, 3, 3>(d, f, W, acc, acc + 6);
      }
    if (d.fn[4])
      for (int j = d.pll_off[g] + threadIdx.x; j < d.pll_off[g + 1]; j += blockDim.x) {
        const int f = d.pll[j];
        T W[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
        for (int64_t i = d.foff[4][f]; i < d.foff[4][f + 1]; ++i) addW_grp<4, T, CD, 3, 4>(d, i, W);
        pair_contrib<T, 3, 4>(d, f, W, acc, acc + 6);
      }
    T* o = block_sum_arr<T, 9>(acc, lds);
    if (threadIdx.x < 9) {
      const int a = threadIdx.x / 3, b = threadIdx.x % 3;
      double v = d.Upl[9 * g + threadIdx.x] + (double)o[sym<3>(a, b)];
      if (a == b) v += lam * d.DA[d.offPl + 3 * g + a];
      d.Spl[9 * g + threadIdx.x] = v;
    }
    if (threadIdx.x < 3) d.bA[d.offPl + 3 * g + threadIdx.x] = -d.gA[d.offPl + 3 * g + threadIdx.x] + (double)o[6 + threadIdx.x];
  } else {
    const int v = blockIdx.x - d.ng;
    T acc[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) acc[k] = 0;
    for (int j = d.vpm_off[v] + threadIdx.x; j < d.vpm_off[v + 1]; j += blockDim.x) {
      const int64_t i = d.vpm[j];
      T W[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
      addW_grp<5, T, CD, 2, 4>(d, i, W);
      pair_contrib<T, 2, 4>(d, d.ffeat[5][i], W, acc, acc + 3);
    }
    T* o = block_sum_arr<T, 5>(acc, lds);
    if (threadIdx.x < 4) {
      const int a = threadIdx.x / 2, b = threadIdx.x % 2;
      double val = d.Uvp[4 * v + threadIdx.x] + (double)o[sym<2>(a, b)];
      if (a == b) val += lam * d.DA[d.offVp + 2 * v + a];
      d.Svp[4 * v + threadIdx.x] = val;
    }
    if (threadIdx.x < 2) d.bA[d.offVp + 2 * v + threadIdx.x] = -d.gA[d.offVp + 2 * v + threadIdx.x] + (double)o[3 + threadIdx.x];
  }
}

void launch_camera_pass_b(const Dev& d, double lambda, hipStream_t s) {
  BA_DISPATCH_T_CD(d, {
    if (d.nc) k_cam_b<T, CD><<<d.nc, 256, 0, s>>>(d, lambda);
    if (d.ng + d.nv) k_grp_b<T, CD><<<d.ng + d.nv, 256, 0, s>>>(d, lambda);
  });
  launch_shape_pass_b(d, lambda, s);
}

// ---------------------------------------------------------------------------
// block-Jacobi preconditioner: M_i = S_ii^-1 (FP64); a block that is not
// positive definite falls back to the inverse of its diagonal
template <int N> __device__ __forceinline__ void invert_block(const double* S, double* M) {
  double A[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) A[i][j] = 0.5 * (S[i * N + j] + S[j * N + i]);
  double Ai[N][N];
  if (chol<double, N>(A)) {
    chol_inverse<double, N>(A, Ai);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) M[i * N + j] = Ai[i][j];
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) M[i * N + j] = (i == j && S[i * N + i] > 0) ? 1.0 / S[i * N + i] : 0.0;
  }
}

template <int CD> __global__ void k_precond_bj(Dev d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.nc) invert_block<CD>(d.Scam + (int64_t)CD * CD * i, d.Mcam + (int64_t)CD * CD * i);
  else if (i < d.nc + d.ng) invert_block<3>(d.Spl + 9 * (i - d.nc), d.Mpl + 9 * (i - d.nc));
  else if (i < d.nc + d.ng + d.nv) invert_block<2>(d.Svp + 4 * (i - d.nc - d.ng), d.Mvp + 4 * (i - d.nc - d.ng));
  else if (i < d.nc + d.ng + d.nv + d.ns) {
    const int q = i - d.nc - d.ng - d.nv;
    invert_block<SH_DOF>(d.Ssh + SH_DOF * SH_DOF * q, d.Msh + SH_DOF * SH_DOF * q);
  }
}

void launch_precond_blockjacobi(const Dev& d, hipStream_t s) {
  const int n = d.nc + d.ng + d.nv + d.ns;
  if (!n) return;
  if (d.CD == 9) k_precond_bj<9><<<nblk(n, 64), 64, 0, s>>>(d);
  else k_precond_bj<6><<<nblk(n, 64), 64, 0, s>>>(d);
}

// ---------------------------------------------------------------------------
// implicit-Schur product y = J_a^T (J_a x - J_f V^-1 J_f^T J_a x) (+ lambda D_a x
// in the reduction), one lane per feature
// One record of the product's first half: q += J_f^T J_a x. The slot is loaded whole,
// except for the surface-group families, whose slots are read a row at a time (ROWS1;
// else all rows' loads at once, where registers allow).
template <int FAM, typename T, int CD, int NF, bool ROWS1 = true>
__device__ __forceinline__ void rec_first(const Dev& d, int64_t i, const T* x, T (&q)[NF]) {
  using SL = Slot<FAM, CD>;
  using F = Fam<FAM, CD>;
  const T* sl = (const T*)d.frec[FAM] + i * SL::STRIDE;
  if constexpr (F::GT == 3) {
    const T* xc = x + CD * d.fcam[FAM][i];
    const T* xg = x + a_grp(d, 3, d.fgrp[FAM][i]);
#pragma unroll ROWS1 ? 1 : SL::ROWS
    for (int row = 0; row < SL::ROWS; ++row) {
      T t = 0;
#pragma unroll
      for (int k = 0; k < SL::NC; ++k) t += sl[SL::OC + row * SL::NC + k] * xc[k];
#pragma unroll
      for (int k = 0; k < SL::NG; ++k) t += sl[SL::OG + row * SL::NG + k] * xg[k];
#pragma unroll
      for (int a = 0; a < NF; ++a) q[a] += sl[SL::OF + row * NF + a] * t;
    }
  } else {
    T v[SL::STRIDE];
    load_vec(sl, v);
    T xc[SL::NC > 0 ? SL::NC : 1], xg[SL::NG > 0 ? SL::NG : 1];
    if constexpr (SL::NC > 0) {
      const T* xp = x + CD * d.fcam[FAM][i];
#pragma unroll
      for (int k = 0; k < SL::NC; ++k) xc[k] = xp[k];
    }
    if constexpr (SL::NG > 0) {
      const T* xp = x + a_grp(d, F::GT, d.fgrp[FAM][i]);
#pragma unroll
      for (int k = 0; k < SL::NG; ++k) xg[k] = xp[k];
    }
#pragma unroll
    for (int row = 0; row < SL::ROWS; ++row) {
      T t = 0;
#pragma unroll
      for (int k = 0; k < SL::NC; ++k) t += v[SL::OC + row * SL::NC + k] * xc[k];
#pragma unroll
      for (int k = 0; k < SL::NG; ++k) t += v[SL::OG + row * SL::NG + k] * xg[k];
#pragma unroll
      for (int a = 0; a < NF; ++a) q[a] += v[SL::OF + row * NF + a] * t;
    }
  }
}

// One record of the second half: y_a += J_a^T (J_a x - J_f s). With gacc, the rows of a
// surface-group record's shape are added to gacc (SH_DOF values) instead of to y.
template <int FAM, typename T, int CD, int NF, bool ROWS1 = true>
__device__ __forceinline__ void rec_second(const Dev& d, int64_t i, const T* x, const T (&s)[NF], double* y, T* gacc = nullptr) {
  using SL = Slot<FAM, CD>;
  using F = Fam<FAM, CD>;
  const T* sl = (const T*)d.frec[FAM] + i * SL::STRIDE;
  int ac = 0, ag = 0;
  if constexpr (SL::NC > 0) ac = CD * d.fcam[FAM][i];
  if constexpr (SL::NG > 0) ag = a_grp(d, F::GT, d.fgrp[FAM][i]);
  T zc[SL::NC > 0 ? SL::NC : 1], zg[SL::NG > 0 ? SL::NG : 1];
#pragma unroll
  for (int k = 0; k < SL::NC; ++k) zc[k] = 0;
#pragma unroll
  for (int k = 0; k < SL::NG; ++k) zg[k] = 0;
  if constexpr (F::GT == 3) {
#pragma unroll ROWS1 ? 1 : SL::ROWS
    for (int row = 0; row < SL::ROWS; ++row) {
      T t = 0;
#pragma unroll
      for (int k = 0; k < SL::NC; ++k) t += sl[SL::OC + row * SL::NC + k] * x[ac + k];
#pragma unroll
      for (int k = 0; k < SL::NG; ++k) t += sl[SL::OG + row * SL::NG + k] * x[ag + k];
#pragma unroll
      for (int a = 0; a < NF; ++a) t -= sl[SL::OF + row * NF + a] * s[a];
#pragma unroll
      for (int k = 0; k < SL::NC; ++k) zc[k] += sl[SL::OC + row * SL::NC + k] * t;
#pragma unroll
      for (int k = 0; k < SL::NG; ++k) zg[k] += sl[SL::OG + row * SL::NG + k] * t;
    }
  } else {
    T v[SL::STRIDE];
    load_vec(sl, v);
    T xc[SL::NC > 0 ? SL::NC : 1], xg[SL::NG > 0 ? SL::NG : 1];
#pragma unroll
    for (int k = 0; k < SL::NC; ++k) xc[k] = x[ac + k];
#pragma unroll
    for (int k = 0; k < SL::NG; ++k) xg[k] = x[ag + k];
#pragma unroll
    for (int row = 0; row < SL::ROWS; ++row) {
      T t = 0;
#pragma unroll
      for (int k = 0; k < SL::NC; ++k) t += v[SL::OC + row * SL::NC + k] * xc[k];
#pragma unroll
      for (int k = 0; k < SL::NG; ++k) t += v[SL::OG + row * SL::NG + k] * xg[k];
#pragma unroll
      for (int a = 0; a < NF; ++a) t -= v[SL::OF + row * NF + a] * s[a];
#pragma unroll
      for (int k = 0; k < SL::NC; ++k) zc[k] += v[SL::OC + row * SL::NC + k] * t;
#pragma unroll
      for (int k = 0; k < SL::NG; ++k) zg[k] += v[SL::OG + row * SL::NG + k] * t;
    }
  }
#pragma unroll
  for (int k = 0; k < SL::NC; ++k) atomicAdd(y + ac + k, (double)zc[k]);
  if constexpr (F::GT == 3) {
    if (gacc) {
#pragma unroll
      for (int k = 0; k < SL::NG; ++k) gacc[k] += zg[k];
      return;
    }
  }
#pragma unroll
  for (int k = 0; k < SL::NG; ++k) atomicAdd(y + ag + k, (double)zg[k]);
}

template <int FAM, typename T, int CD, int NF> __device__ __forceinline__ void mv_first(const Dev& d, int f, const T* x, T (&q)[NF]) {
  if (!d.fn[FAM]) return;
  for (int64_t i = d.foff[FAM][f]; i < d.foff[FAM][f + 1]; ++i) rec_first<FAM, T, CD, NF>(d, i, x, q);
}

template <int FAM, typename T, int CD, int NF> __device__ __forceinline__ void mv_second(const Dev& d, int f, const T* x, const T (&s)[NF], double* y) {
  if (!d.fn[FAM]) return;
  for (int64_t i = d.foff[FAM][f]; i < d.foff[FAM][f + 1]; ++i) rec_second<FAM, T, CD, NF>(d, i, x, s, y);
}

// One wavefront per feature (a feature larger than a tile, or a line on a shape): its
// records, family after family, over the lanes in rounds of 64; q summed across the
// wavefront, s_f solved on every lane, then each lane's records added to y. The shape
// rows (a feature is on one shape at most) are summed across the wavefront and added
// once. Every lane of the wavefront calls this with the same f, and all are active.
template <int FAM, typename T, int CD, int NF>
__device__ __forceinline__ void wave_first(const Dev& d, int64_t b, int n, const T* x, int& j0, int lane, T (&q)[NF]) {
  // the family's records continue the feature's sequence at position j0: record r is on
  // lane (j0 + r) mod 64
  for (int r = (lane - j0 % 64 + 64) % 64; r < n; r += 64) rec_first<FAM, T, CD, NF, false>(d, b + r, x, q);
  j0 += n;
}

template <int FAM, typename T, int CD, int NF>
__device__ __forceinline__ void wave_second(const Dev& d, int64_t b, int n, const T* x, const T (&s)[NF], double* y,
                                            int& j0, int lane, T* gacc = nullptr) {
  for (int r = (lane - j0 % 64 + 64) % 64; r < n; r += 64) rec_second<FAM, T, CD, NF, false>(d, b + r, x, s, y, gacc);
  j0 += n;
}

// shy: when given, the shape rows go to this LDS copy of y's shape block (index from
// d.offSh) instead of to y
template <typename T, int CD, int NF>
__device__ __forceinline__ void mv_feature_wave(const Dev& d, int f, const T* x, double* y, int lane, double* shy = nullptr) {
  constexpr int F0 = NF == 3 ? 1 : 2, F1 = NF == 3 ? 3 : 4, F2 = NF == 3 ? 6 : 5, F3 = NF == 3 ? 8 : 7;
  constexpr int FS = NF == 3 ? 9 : 10, NS = NF * (NF + 1) / 2;
  // every family's record range, the feature's inverse and flag fetched together (one
  // memory round ahead of the records), then the shape's rows in y
  int64_t b[5];
  int n[5];
  auto range = [&](int k, int F) {
    if (d.fn[F]) {
      b[k] = d.foff[F][f];
      n[k] = (int)(d.foff[F][f + 1] - b[k]);
    } else {
      b[k] = 0;
      n[k] = 0;
    }
  };
  range(0, F0); range(1, F1); range(2, F2); range(3, F3); range(4, FS);
  const bool flag = (NF == 3 ? d.flp : d.fll)[f] != 0;
  T m[NS];
  {
    const T* M = (const T*)(NF == 3 ? d.Vip : d.Vil) + (int64_t)NS * f;
#pragma unroll
    for (int k = 0; k < NS; ++k) m[k] = M[k];
  }
  const int ag = n[4] > 0 ? a_grp(d, 3, d.fgrp[FS][b[4]]) : 0;
  T q[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) q[k] = 0;
  int j0 = 0;
  wave_first<F0, T, CD, NF>(d, b[0], n[0], x, j0, lane, q);
  wave_first<F1, T, CD, NF>(d, b[1], n[1], x, j0, lane, q);
  wave_first<F2, T, CD, NF>(d, b[2], n[2], x, j0, lane, q);
  wave_first<F3, T, CD, NF>(d, b[3], n[3], x, j0, lane, q);
  wave_first<FS, T, CD, NF>(d, b[4], n[4], x, j0, lane, q);
#pragma unroll
  for (int k = 0; k < NF; ++k) q[k] = wave_sum(q[k]);
  T s[NF];
  if (flag) {
    apply_vinv<T, NF>(d, f, q, s);  // a flagged block: its FP64 inverse
  } else {
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      T t = 0;
#pragma unroll
      for (int j = 0; j < NF; ++j) t += m[sym<NF>(i, j)] * q[j];
      s[i] = t;
    }
  }
  // the second half's records in any order: the shape's first, so that their sums are
  // added (and released) before the other families' records
  j0 = 0;
  if (n[4] > 0) {
    T gacc[SH_DOF];
#pragma unroll
    for (int k = 0; k < SH_DOF; ++k) gacc[k] = 0;
    wave_second<FS, T, CD, NF>(d, b[4], n[4], x, s, y, j0, lane, gacc);
    double* ys = shy ? shy + (ag - d.offSh) : y + ag;
#pragma unroll
    for (int k = 0; k < SH_DOF; ++k) {
      const T w = wave_sum(gacc[k]);
      if (lane == 0) atomicAdd(ys + k, (double)w);
    }
  }
  wave_second<F0, T, CD, NF>(d, b[0], n[0], x, s, y, j0, lane);
  wave_second<F1, T, CD, NF>(d, b[1], n[1], x, s, y, j0, lane);
  wave_second<F2, T, CD, NF>(d, b[2], n[2], x, s, y, j0, lane);
  wave_second<F3, T, CD, NF>(d, b[3], n[3], x, s, y, j0, lane);
}

// deterministic product, first pass: s_f = (V_f + lambda D_f)^-1 J_f^T J_a x of one feature
template <typename T, int CD, int NF> __device__ __forceinline__ void mv_feature_s(const Dev& d, int f, const T* x) {
  T q[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) q[k] = 0;
  if constexpr (NF == 3) {
    mv_first<1, T, CD, 3>(d, f, x, q);
    mv_first<3, T, CD, 3>(d, f, x, q);
    mv_first<6, T, CD, 3>(d, f, x, q);
    mv_first<8, T, CD, 3>(d, f, x, q);
    mv_first<9, T, CD, 3>(d, f, x, q);
  } else {
    mv_first<2, T, CD, 4>(d, f, x, q);
    mv_first<4, T, CD, 4>(d, f, x, q);
    mv_first<5, T, CD, 4>(d, f, x, q);
    mv_first<7, T, CD, 4>(d, f, x, q);
    mv_first<10, T, CD, 4>(d, f, x, q);
  }
  T sv[NF];
  apply_vinv<T, NF>(d, f, q, sv);
  T* o = (T*)(NF == 3 ? d.sdp : d.sdl) + (int64_t)NF * f;
#pragma unroll
  for (int k = 0; k < NF; ++k) o[k] = sv[k];
}

// ---------------------------------------------------------------------------
// Wavefront-tiled implicit-Schur product.  A tile is a run of consecutive
// features (points, or lines) with at most 64 records over all their families,
// stored as one packed (family, record) word per lane in feature order.  Each
// wavefront takes its own tiles, one record per lane, with no workgroup barrier:
//   A  t = J_a x;  q_f = sum of J_f^T t over the feature's lanes (segmented
//      scan across the wavefront; the feature's last lane holds the sum)
//   B  s_f = (V_f + lambda D_f)^-1 q_f on that last lane, broadcast to the
//      feature's lanes
//   C  u = t - J_f s_f;  y_a += J_a^T u   (FP64 LDS atomics into the
//      workgroup's y, which all its wavefronts share)
// Each workgroup writes its y to its row of the partial buffer.
template <int CD> struct MaxSlot { static constexpr int V = Slot<4, CD>::STRIDE; };
static_assert(Slot<9, 9>::STRIDE <= MaxSlot<9>::V && Slot<9, 6>::STRIDE <= MaxSlot<6>::V,
              "point-on-shape records fit the tiles' register slot");

template <int FAM, typename T, int CD>
__device__ __forceinline__ void tile_phase_a(const Dev& d, int64_t i, int cam, int grp, const T* x, T (&qv)[4],
                                             T (&v)[MaxSlot<CD>::V], T (&t)[4], int& ac, int& ag) {
  using SL = Slot<FAM, CD>;
  using F = Fam<FAM, CD>;
  const T* rec = (const T*)d.frec[FAM] + i * SL::STRIDE;
  if constexpr (sizeof(T) == 4) {
    const float4* q4 = reinterpret_cast<const float4*>(rec);
#pragma unroll
    for (int k = 0; k < SL::STRIDE / 4; ++k) {
      float4 a = q4[k];
      v[4 * k] = a.x; v[4 * k + 1] = a.y; v[4 * k + 2] = a.z; v[4 * k + 3] = a.w;
    }
  } else {
    const double2* q2 = reinterpret_cast<const double2*>(rec);
#pragma unroll
    for (int k = 0; k < SL::STRIDE / 2; ++k) {
      double2 a = q2[k];
      v[2 * k] = a.x; v[2 * k + 1] = a.y;
    }
  }
  if constexpr (SL::NC > 0) ac = CD * cam;
  if constexpr (SL::NG > 0) ag = a_grp(d, F::GT, grp);
  T xc[SL::NC > 0 ? SL::NC : 1], xg[SL::NG > 0 ? SL::NG : 1];
#pragma unroll
  for (int k = 0; k < SL::NC; ++k) xc[k] = x[ac + k];
#pragma unroll
  for (int k = 0; k < SL::NG; ++k) xg[k] = x[ag + k];
#pragma unroll
  for (int row = 0; row < SL::ROWS; ++row) {
    T tt = 0;
#pragma unroll
    for (int k = 0; k < SL::NC; ++k) tt += v[SL::OC + row * SL::NC + k] * xc[k];
#pragma unroll
    for (int k = 0; k < SL::NG; ++k) tt += v[SL::OG + row * SL::NG + k] * xg[k];
    t[row] = tt;
  }
#pragma unroll
  for (int a = 0; a < SL::NF; ++a) {
    T qa = 0;
#pragma unroll
    for (int row = 0; row < SL::ROWS; ++row) qa += v[SL::OF + row * SL::NF + a] * t[row];
    qv[a] = qa;
  }
}

// sum of v over the 64 lanes of a wavefront whose lanes are all active, the same on every
// lane: xor exchanges within each half by ds_swizzle (its lane pattern is an immediate,
// so no address register is held), then the two halves' sums read from lanes 0 and 32
__device__ __forceinline__ float wave_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (1 << 10)));
  v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (2 << 10)));
  v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (4 << 10)));
  v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (8 << 10)));
  v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (16 << 10)));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0)) +
         __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
}

template <int XOR> __device__ __forceinline__ double swizzle_xor(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffffll), 0x1F | (XOR << 10));
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x1F | (XOR << 10));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_sum(double v) {
  v += swizzle_xor<1>(v);
  v += swizzle_xor<2>(v);
  v += swizzle_xor<4>(v);
  v += swizzle_xor<8>(v);
  v += swizzle_xor<16>(v);
  const long long b = __double_as_longlong(v);
  const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  const double h0 = __longlong_as_double(((long long)__builtin_amdgcn_readlane(hi, 0) << 32) |
                                         (unsigned int)__builtin_amdgcn_readlane(lo, 0));
  const double h1 = __longlong_as_double(((long long)__builtin_amdgcn_readlane(hi, 32) << 32) |
                                         (unsigned int)__builtin_amdgcn_readlane(lo, 32));
  return h0 + h1;
}

// In FP32 the shape rows (group type 3) are staged in the wavefront's LDS rows gz[k *
// 64] for the wavefront's sum after the tile (a tile's lanes are mostly points of one
// shape); every other row is added to y here.
template <int FAM, typename T, int CD>
__device__ __forceinline__ void tile_phase_c(const T (&v)[MaxSlot<CD>::V], const T (&t)[4], int ac, int ag,
                                             const T (&sv)[4], double* y, T* gz) {
  using SL = Slot<FAM, CD>;
  constexpr bool WAVE_G = Fam<FAM, CD>::GT == 3 && sizeof(T) == 4;
  static_assert(!WAVE_G || SL::NG == SH_DOF, "shape rows");
  T zc[SL::NC > 0 ? SL::NC : 1], zg[SL::NG > 0 ? SL::NG : 1];
#pragma unroll
  for (int k = 0; k < SL::NC; ++k) zc[k] = 0;
#pragma unroll
  for (int k = 0; k < SL::NG; ++k) zg[k] = 0;
#pragma unroll
  for (int row = 0; row < SL::ROWS; ++row) {
    T u = t[row];
#pragma unroll
    for (int a = 0; a < SL::NF; ++a) u -= v[SL::OF + row * SL::NF + a] * sv[a];
#pragma unroll
    for (int k = 0; k < SL::NC; ++k) zc[k] += v[SL::OC + row * SL::NC + k] * u;
#pragma unroll
    for (int k = 0; k < SL::NG; ++k) zg[k] += v[SL::OG + row * SL::NG + k] * u;
  }
#pragma unroll
  for (int k = 0; k < SL::NC; ++k) atomicAdd(y + ac + k, (double)zc[k]);
  if constexpr (WAVE_G) {
#pragma unroll
    for (int k = 0; k < SH_DOF; ++k) gz[k * 64] = zg[k];
  } else {
#pragma unroll
    for (int k = 0; k < SL::NG; ++k) atomicAdd(y + ag + k, (double)zg[k]);
  }
}

// FP64 records are reloaded for phase C instead of being held in registers
template <int FAM, typename T, int CD>
__device__ __forceinline__ void tile_phase_c_reload(const Dev& d, int64_t i, const T (&t)[4], int ac, int ag,
                                                    const T (&sv)[4], double* y, T* gz) {
  using SL = Slot<FAM, CD>;
  T v[MaxSlot<CD>::V];
  const double2* q2 = reinterpret_cast<const double2*>((const T*)d.frec[FAM] + i * SL::STRIDE);
#pragma unroll
  for (int k = 0; k < SL::STRIDE / 2; ++k) {
    double2 a = q2[k];
    v[2 * k] = a.x; v[2 * k + 1] = a.y;
  }
  tile_phase_c<FAM, T, CD>(v, t, ac, ag, sv, y, gz);
}

// s = (V_f + lambda D_f)^-1 q for feature f from its packed FP32 inverse Mi, or
// the FP64 one of a flagged block
template <typename T, int NF>
__device__ __forceinline__ void feature_solve(const Dev& d, int f, bool flag, const T (&Mi)[10], const T (&q)[4], T (&s)[4]) {
  T qn[NF], sn[NF];
#pragma unroll
  for (int a = 0; a < NF; ++a) qn[a] = q[a];
  if (flag) {
    apply_vinv<T, NF>(d, f, qn, sn);
  } else {
#pragma unroll
    for (int a = 0; a < NF; ++a) {
      T acc = 0;
#pragma unroll
      for (int b = 0; b < NF; ++b) acc += Mi[sym<NF>(a, b)] * qn[b];
      sn[a] = acc;
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) s[a] = a < NF ? sn[a] : T(0);
}

// With SONLY (the deterministic mode's first pass) a tile stops after B: the feature's
// last lane stores s_f (d.sdp / d.sdl) and nothing is added to y.
template <typename T, int CD, bool LDSY, bool SONLY = false>
__global__ __launch_bounds__(MV_THREADS) void k_mv_wave(Dev d, const double* done) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (done && *done != 0.0) return;
  double* ys = LDSY ? reinterpret_cast<double*>(smem_raw) : d.mv_part;
  // FP32 shape rows staged per lane (column lane of the wavefront's SH_DOF x 64 rows),
  // and the lane's shape offset in y (-1: not a shape record), after y in LDS; present
  // when d.mv_stage (then every tile writes its offsets). A lane reads back only what it
  // wrote, and nothing of it stays in registers across the record phases.
  constexpr bool STAGE = sizeof(T) == 4 && !SONLY;
  const bool stage = STAGE && d.mv_stage;
  float* mv_stage = reinterpret_cast<float*>(smem_raw + (LDSY ? 8 * (size_t)d.nA : 0));
  int* mv_shag = reinterpret_cast<int*>(mv_stage + MV_THREADS / 64 * SH_DOF * 64);
  const T* x = (const T*)d.xT;
  if constexpr (LDSY) {
    for (int k = threadIdx.x; k < d.nA; k += blockDim.x) ys[k] = 0;
    __syncthreads();
  }
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int tile = blockIdx.x * nw + (threadIdx.x >> 6); tile < d.n_tiles; tile += gridDim.x * nw) {
    const int4 tl = d.tiles[tile];  // (first slot, slots, first feature, -)
    const int fb = tl.z;
    const bool active = lane < tl.y;
    const bool ptile = tile < d.n_ptiles;
    int4 w4 = make_int4(0, 0, 0, -1);
    if (active) w4 = d.wrec[tl.x + lane];
    const int fam = (int)((uint32_t)w4.x >> 28), lf = w4.w;
    const int64_t i = (int64_t)((uint32_t)w4.x & 0x0fffffffu);
    // the feature's last lane solves with its inverse: fetched now, beside the record
    const int next = __shfl_down(lf, 1, 64);
    const bool last = lf >= 0 && (lane == 63 || next != lf);
    T Mi[10];
    bool mflag = false;
    if (last) {
      const int f = fb + lf;
      mflag = (ptile ? d.flp[f] : d.fll[f]) != 0;
      if (ptile) {
        const T* M = (const T*)d.Vip + 6 * (int64_t)f;
#pragma unroll
        for (int k = 0; k < 6; ++k) Mi[k] = M[k];
      } else {
        const T* M = (const T*)d.Vil + 10 * (int64_t)f;
#pragma unroll
        for (int k = 0; k < 10; ++k) Mi[k] = M[k];
      }
    }
    T v[MaxSlot<CD>::V];
    T t[4] = {0, 0, 0, 0};
    T q[4] = {0, 0, 0, 0};
    int ac = 0, ag = 0;
    if (active) {
      switch (fam) {
        case 1: tile_phase_a<1, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 2: tile_phase_a<2, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 3: tile_phase_a<3, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 4: tile_phase_a<4, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 5: tile_phase_a<5, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 6: tile_phase_a<6, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 7: tile_phase_a<7, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 8: tile_phase_a<8, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 9: tile_phase_a<9, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
      }
    }
    // segmented inclusive scan over runs of equal lf (lanes are in feature
    // order; inactive lanes, lf = -1, come last); a lane adds the value `off`
    // lanes back while that lane is in its run
    const int prev = __shfl_up(lf, 1, 64);
    const unsigned long long heads = __ballot(lf >= 0 && (lane == 0 || prev != lf));
    const int start = lf >= 0 ? 63 - __builtin_clzll(heads & ((2ull << lane) - 1ull)) : lane;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const bool take = lane - off >= start;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (a == 3 && ptile) continue;  // points have 3 components
        const T o = __shfl_up(q[a], off, 64);
        if (take) q[a] += o;
      }
    }
    const unsigned long long lasts = __ballot(last);
    T s[4] = {0, 0, 0, 0};
    if (last) {
      if (ptile) feature_solve<T, 3>(d, fb + lf, mflag, Mi, q, s);
      else feature_solve<T, 4>(d, fb + lf, mflag, Mi, q, s);
    }
    if constexpr (SONLY) {
      if (last) {
        if (ptile) {
          T* o = (T*)d.sdp + 3 * (int64_t)(fb + lf);
          o[0] = s[0]; o[1] = s[1]; o[2] = s[2];
        } else {
          T* o = (T*)d.sdl + 4 * (int64_t)(fb + lf);
          o[0] = s[0]; o[1] = s[1]; o[2] = s[2]; o[3] = s[3];
        }
      }
      continue;
    }
    if (stage) mv_shag[threadIdx.x] = active && fam == 9 ? ag : -1;
    const int src = lf >= 0 ? __builtin_ctzll(lasts & (~0ull << lane)) : lane;
#pragma unroll
    for (int a = 0; a < 4; ++a) s[a] = __shfl(s[a], src, 64);
    if (active) {
      if constexpr (sizeof(T) == 4) {
        switch (fam) {
          case 1: tile_phase_c<1, T, CD>(v, t, ac, ag, s, ys, nullptr); break;
          case 2: tile_phase_c<2, T, CD>(v, t, ac, ag, s, ys, nullptr); break;
          case 3: tile_phase_c<3, T, CD>(v, t, ac, ag, s, ys, nullptr); break;
          case 4: tile_phase_c<4, T, CD>(v, t, ac, ag, s, ys, nullptr); break;
          case 5: tile_phase_c<5, T, CD>(v, t, ac, ag, s, ys, nullptr); break;
          case 6: tile_phase_c<6, T, CD>(v, t, ac, ag, s, ys, nullptr); break;
          case 7: tile_phase_c<7, T, CD>(v, t, ac, ag, s, ys, nullptr); break;
          case 8: tile_phase_c<8, T, CD>(v, t, ac, ag, s, ys, nullptr); break;
          case 9: tile_phase_c<9, T, CD>(v, t, ac, ag, s, ys, reinterpret_cast<T*>(mv_stage) + (threadIdx.x >> 6) * SH_DOF * 64 + lane); break;
        }
      } else {
        switch (fam) {
          case 1: tile_phase_c_reload<1, T, CD>(d, i, t, ac, ag, s, ys, nullptr); break;
          case 2: tile_phase_c_reload<2, T, CD>(d, i, t, ac, ag, s, ys, nullptr); break;
          case 3: tile_phase_c_reload<3, T, CD>(d, i, t, ac, ag, s, ys, nullptr); break;
          case 4: tile_phase_c_reload<4, T, CD>(d, i, t, ac, ag, s, ys, nullptr); break;
          case 5: tile_phase_c_reload<5, T, CD>(d, i, t, ac, ag, s, ys, nullptr); break;
          case 6: tile_phase_c_reload<6, T, CD>(d, i, t, ac, ag, s, ys, nullptr); break;
          case 7: tile_phase_c_reload<7, T, CD>(d, i, t, ac, ag, s, ys, nullptr); break;
          case 8: tile_phase_c_reload<8, T, CD>(d, i, t, ac, ag, s, ys, nullptr); break;
          case 9: tile_phase_c_reload<9, T, CD>(d, i, t, ac, ag, s, ys, nullptr); break;
        }
      }
    }
    // FP32 shape rows: the lanes on the wavefront's first shape are summed across it and
    // added once (one LDS add per row, not one per record on the same address); lanes on
    // another shape add their own. A lane reads back only what it staged itself.
    if (stage) {
      const int shag = mv_shag[threadIdx.x];
      const unsigned long long gm = __ballot(shag >= 0);
      if (gm) {
        const int l = threadIdx.x & 63, lead = __builtin_ctzll(gm);
        const int ag0 = __builtin_amdgcn_readlane(shag, lead);
        const bool mine = shag == ag0;
        const float* gst = mv_stage + (threadIdx.x >> 6) * SH_DOF * 64 + l;
#pragma unroll
        for (int k = 0; k < SH_DOF; ++k) {
          const float w = wave_sum(mine ? gst[k * 64] : 0.0f);
          if (l == lead) atomicAdd(ys + ag0 + k, (double)w);
        }
        if (shag >= 0 && !mine)
#pragma unroll
          for (int k = 0; k < SH_DOF; ++k) atomicAdd(ys + shag + k, (double)gst[k * 64]);
      }
    }
  }
  // features whose records do not fit one tile (and the lines on a shape) are k_mv_big's;
  // the deterministic mode's first pass takes them here, one lane each, dealt round-robin
  // over the workgroups (lane t of workgroup b takes b + t * gridDim.x)
  if constexpr (SONLY) {
    for (int k = blockIdx.x + gridDim.x * threadIdx.x; k < d.n_bigp + d.n_bigl; k += gridDim.x * blockDim.x) {
      if (k < d.n_bigp) mv_feature_s<T, CD, 3>(d, d.bigp[k], x);
      else mv_feature_s<T, CD, 4>(d, d.bigl[k - d.n_bigp], x);
    }
  }
  if constexpr (LDSY) {
    __syncthreads();
    double* out = d.mv_part + (int64_t)blockIdx.x * d.nA;
    for (int k = threadIdx.x; k < d.nA; k += blockDim.x) out[k] = ys[k];
  }
}

// The product's features larger than a tile (and the lines on a shape), one wavefront
// each, launched after k_mv_wave on its stream: FP64 global atomics into row 0 of the
// product partials, which k_mv_wave has written (LDS y) or accumulated into (global y).
// A kernel of its own, so that its registers do not add to the tiles'; run alone, so that
// its chain of dependent memory rounds is not slowed by the tiles' traffic (measured
// slower beside them on a second stream).
template <typename T, int CD> __global__ __launch_bounds__(MV_BIG_THREADS) void k_mv_big(Dev d, const double* done) {
  // the shape rows summed in LDS first and added to y once per workgroup (the features of
  // one shape would otherwise all add into the same global rows, one after another)
  extern __shared__ double big_sh[];
  if (done && *done != 0.0) return;
  const bool lsh = d.ns > 0 && d.ns * SH_DOF <= MV_BIG_SH_MAX;
  if (lsh) {
    for (int k = threadIdx.x; k < d.ns * SH_DOF; k += blockDim.x) big_sh[k] = 0;
    __syncthreads();
  }
  const T* x = (const T*)d.xT;
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int k = blockIdx.x * nw + (threadIdx.x >> 6); k < d.n_bigp + d.n_bigl; k += gridDim.x * nw) {
    if (k < d.n_bigp) mv_feature_wave<T, CD, 3>(d, d.bigp[k], x, d.mv_part, lane, lsh ? big_sh : nullptr);
    else mv_feature_wave<T, CD, 4>(d, d.bigl[k - d.n_bigp], x, d.mv_part, lane, lsh ? big_sh : nullptr);
  }
  if (lsh) {
    __syncthreads();
    for (int k = threadIdx.x; k < d.ns * SH_DOF; k += blockDim.x)
      if (big_sh[k] != 0.0) atomicAdd(d.mv_part + d.offSh + k, big_sh[k]);
  }
}

template <typename T> __global__ void k_to_T(const double* src, void* dst, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) ((T*)dst)[k] = (T)src[k];
}

int matvec_max_lds_bytes() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 65536;
  return v;
}

size_t matvec_lds_bytes(const Dev& d) { return (d.mv_lds ? 8 * (size_t)d.nA : 0) + (d.mv_stage ? MV_STAGE_BYTES : 0); }

template <typename T, int CD, bool LDSY> static void launch_mv(const Dev& d, const double* done, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    // on failure the launch below reports the LDS request through the launch check
    attr = hipFuncSetAttribute((const void*)k_mv_wave<T, CD, LDSY>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               matvec_max_lds_bytes()) == hipSuccess;
  }
  k_mv_wave<T, CD, LDSY><<<d.n_mv_wg, MV_THREADS, matvec_lds_bytes(d), s>>>(d, done);
  const int nbig = d.n_bigp + d.n_bigl;
  if (nbig) {
    const size_t sh = d.ns > 0 && d.ns * SH_DOF <= MV_BIG_SH_MAX ? (size_t)d.ns * SH_DOF * sizeof(double) : 0;
    k_mv_big<T, CD><<<std::min(nblk(nbig, MV_BIG_THREADS / 64), 4096u), MV_BIG_THREADS, sh, s>>>(d, done);
  }
}

// deterministic product, second pass (defined with the S Z sweeps, whose record and
// block-sum helpers it shares): every row of y from its records in a fixed order
template <typename T, int CD> void launch_det_rows(const Dev& d, const double* done, hipStream_t s);

template <typename T, int CD> static void run_matvec(const Dev& d, const double* done, hipStream_t s) {
  if (d.det) {
    k_mv_wave<T, CD, false, true><<<d.n_mv_wg, MV_THREADS, 0, s>>>(d, done);
    launch_det_rows<T, CD>(d, done, s);
  } else if (d.mv_lds) {
    launch_mv<T, CD, true>(d, done, s);
  } else {
    launch_mv<T, CD, false>(d, done, s);
  }
  launch_rel_matvec(d, done, s);  // the inter-group relations' rows, added by k_pcg_q
}

// ---------------------------------------------------------------------------
// PCG vector kernels, grid-wide.  Dot products are summed with one FP64
// atomic per workgroup into accumulator set k mod 3 of iteration k; the next
// kernel on the stream reads the sum.  Iteration k zeroes set (k + 1) mod 3,
// whose last reader ran in iteration k - 2.
__device__ __forceinline__ double* acc_set(const Dev& d, int k) { return d.scal + SC_ACC + ACC_STRIDE * (k % 3); }

// position of entry e of the reduced vector: its block's offset, size and preconditioner block
template <int CD> __device__ __forceinline__ void entry_block(const Dev& d, int e, int& o, int& n, const double*& M) {
  if (e < d.offPl) { const int b = e / CD; o = CD * b; n = CD; M = d.Mcam + (int64_t)CD * CD * b; }
  else if (e < d.offVp) { const int g = (e - d.offPl) / 3; o = d.offPl + 3 * g; n = 3; M = d.Mpl + 9 * g; }
  else if (e < d.offSh) { const int v = (e - d.offVp) / 2; o = d.offVp + 2 * v; n = 2; M = d.Mvp + 4 * v; }
  else { const int q = (e - d.offSh) / SH_DOF; o = d.offSh + SH_DOF * q; n = SH_DOF; M = d.Msh + SH_DOF * SH_DOF * q; }
}

// Accumulator slot of dst (a scalar of d.scal, or an entry of Z^T b) in the deterministic
// mode's partial table
__device__ __forceinline__ int64_t det_slot(const Dev& d, const double* dst) {
  const int64_t k = dst - d.scal;
  return (k >= 0 && k < SC_COUNT) ? k : SC_COUNT + (dst - d.Ztb);
}

// add this workgroup's sum v to the accumulator dst: one FP64 atomic, or in the
// deterministic mode the workgroup's entry of the partial table (k_det_sum adds them in
// workgroup order)
__device__ __forceinline__ void acc_add(const Dev& d, double* dst, double v) {
  if (d.det) d.detp[det_slot(d, dst) * d.det_stride + blockIdx.x] = v;
  else atomicAdd(dst, v);
}

// deterministic mode: accumulators [lo, lo + n) and [lo2, lo2 + n2) (slot numbers as in
// det_slot) = the sum of their nwg workgroup partials, in workgroup order.  Skipped when
// the PCG has stopped, like the kernels that write the partials.
__global__ void k_det_sum(Dev d, int lo, int n, int lo2, int n2, int nwg) {
  if (d.scal[SC_DONE] != 0.0 || d.scal[SC_BREAK] != 0.0) return;
  const int t = threadIdx.x;
  const int slot = t < n ? lo + t : t < n + n2 ? lo2 + (t - n) : -1;
  if (slot < 0) return;
  const double* p = d.detp + (int64_t)slot * d.det_stride;
  double s = 0;
  for (int w = 0; w < nwg; ++w) s += p[w];
  if (slot < SC_COUNT) d.scal[slot] = s;
  else d.Ztb[slot - SC_COUNT] = s;
}

// one FP64 atomic (or deterministic partial) per workgroup for each of K block sums
template <int K> __device__ __forceinline__ void block_atomic_add(const Dev& d, double (&v)[K], double* lds,
                                                                  double* const (&dst)[K]) {
  double* o = block_sum_arr<double, K>(v, lds);
  if (threadIdx.x < K) acc_add(d, dst[threadIdx.x], o[threadIdx.x]);
}

// ---- two-level preconditioner (coarse space Z, E = Z^T S Z) -----------------
// y = E^-1 v for the active columns (every thread computes it; K <= 15)
__device__ __forceinline__ void coarse_solve(const Dev& d, const double* v, double (&y)[COARSE_K]) {
  const int K = d.coarse_k;
  for (int a = 0; a < COARSE_K; ++a) {
    double t = 0;
    if (a < K)
      for (int b = 0; b < K; ++b) t += d.Einv[a * COARSE_K + b] * v[b];
    y[a] = t;
  }
}

// sum_c Z[c][e] y_c
__device__ __forceinline__ double coarse_combine(const Dev& d, int e, const double (&y)[COARSE_K]) {
  double t = 0;
  for (int c = 0; c < d.coarse_k; ++c) t += d.Zc[(int64_t)c * d.nA + e] * y[c];
  return t;
}

// full r.z of iteration set A: r.(M r) + (Z^T r) . E^-1 (Z^T r - (S Z)^T M r)
__device__ __forceinline__ double coarse_rz(const Dev& d, const double* A, double (&y)[COARSE_K]) {
  double v[COARSE_K];
  for (int c = 0; c < COARSE_K; ++c) v[c] = c < d.coarse_k ? A[ACC_ZR + c] - A[ACC_W + c] : 0.0;
  coarse_solve(d, v, y);
  double rz = A[ACC_RZ];
  for (int c = 0; c < d.coarse_k; ++c) rz += A[ACC_ZR + c] * y[c];
  return rz;
}


// Ztb = Z^T b (Ztb cleared by k_pcg_reset)
__global__ __launch_bounds__(256) void k_coarse_ztb(Dev d) {
  __shared__ double lds[5 * COARSE_K];
  if (d.scal[SC_COARSE] == 0.0) return;
  double v[COARSE_K];
  for (int a = 0; a < COARSE_K; ++a) v[a] = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < d.nA; e += gridDim.x * blockDim.x) {
    const double be = d.bA[e];
    for (int a = 0; a < d.coarse_k; ++a) v[a] += d.Zc[(int64_t)a * d.nA + e] * be;
  }
  double* o = block_sum_arr<double, COARSE_K>(v, lds);
  if (threadIdx.x < d.coarse_k) acc_add(d, d.Ztb + threadIdx.x, o[threadIdx.x]);
}

// coarse start: u = E^-1 Z^T b, x0 = Z u, r0 = b - (S Z) u, z = M r0 (stored in d.z);
// set 2 gets r0.(M r0), Z^T r0 and (S Z)^T M r0; b.b -> SC_BB   (one thread per entry)
template <int CD> __global__ __launch_bounds__(256) void k_pcg_init_coarse(Dev d) {
  constexpr int NV = 2 + 2 * COARSE_K;
  __shared__ double lds[5 * NV];
  const bool on = d.coarse_k > 0 && d.scal[SC_COARSE] != 0.0;
  double u[COARSE_K];
  if (on) coarse_solve(d, d.Ztb, u);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0;
  if (e < d.nA) {
    int o, n;
    const double* M;
    entry_block<CD>(d, e, o, n, M);
    const int row = e - o;
    auto r0 = [&](int j) {  // b - S Z u at entry j
      double t = d.bA[j];
      if (on)
        for (int c = 0; c < d.coarse_k; ++c) t -= d.SZc[(int64_t)c * d.nA + j] * u[c];
      return t;
    };
    const double re = r0(e);
    double zm = 0;
    for (int c = 0; c < n; ++c) zm += M[row * n + c] * r0(o + c);
    d.x[e] = on ? coarse_combine(d, e, u) : 0.0;
    d.r[e] = re;
    d.z[e] = zm;
    v[0] = re * zm;
    v[1] = d.bA[e] * d.bA[e];
    if (on)
      for (int c = 0; c < d.coarse_k; ++c) {
        v[2 + c] = d.Zc[(int64_t)c * d.nA + e] * re;
        v[2 + COARSE_K + c] = d.SZc[(int64_t)c * d.nA + e] * zm;
      }
  }
  double* A = acc_set(d, 2);
  double* o2 = block_sum_arr<double, NV>(v, lds);
  if (threadIdx.x < NV) {
    const int k = threadIdx.x;
    double* dst = k == 0 ? A + ACC_RZ : k == 1 ? d.scal + SC_BB : k < 2 + COARSE_K ? A + ACC_ZR + (k - 2) : A + ACC_W + (k - 2 - COARSE_K);
    acc_add(d, dst, o2[k]);
  }
}

// p = z = M r0 + Z E^-1 (Z^T r0 - (S Z)^T M r0)   (one thread per entry)
template <typename T> __global__ __launch_bounds__(256) void k_pcg_init_coarse2(Dev d) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d.nA) return;
  double z = d.z[e];
  if (d.coarse_k > 0 && d.scal[SC_COARSE] != 0.0) {
    double y[COARSE_K];
    coarse_rz(d, acc_set(d, 2), y);
    z += coarse_combine(d, e, y);
  }
  d.z[e] = z;
  d.p[e] = z;
  ((T*)d.xT)[e] = (T)z;
}

// scalars of a new solve: accumulators cleared, tolerances set (one thread)
__global__ void k_pcg_reset(Dev d, double tol, int maxit) {
  for (int k = 0; k < 3 * ACC_STRIDE; ++k) d.scal[SC_ACC + k] = 0;
  if (d.Ztb)
    for (int k = 0; k < COARSE_K; ++k) d.Ztb[k] = 0;
  d.scal[SC_BB] = 0;
  d.scal[SC_ITER] = 0;
  d.scal[SC_MAXIT] = maxit;
  d.scal[SC_BREAK] = 0;
  d.scal[SC_DONE] = 0;
  d.scal[SC_TOL2] = tol * tol;  // scaled by b.b in k_pcg_start
}

__global__ void k_pcg_start(Dev d) {
  const double bb = d.scal[SC_BB];
  d.scal[SC_RR] = bb;
  double rz = acc_set(d, 2)[ACC_RZ];
  if (d.coarse_k > 0 && d.scal[SC_COARSE] != 0.0) {
    double y[COARSE_K];
    rz = coarse_rz(d, acc_set(d, 2), y);
  }
  d.scal[SC_RZ] = rz;
  d.scal[SC_TOL2] *= bb;
  if (bb == 0.0 || d.scal[SC_MAXIT] <= 0 || !isfinite(bb)) d.scal[SC_DONE] = 1.0;
}

// q = sum of the product partials + lambda D p; p.q -> set k
// workgroup: 64 entries x 16 partial slices
template <typename T> __global__ __launch_bounds__(1024) void k_pcg_q(Dev d, const double* done, const double* xin,
                                                                     double* y, double lam, int k) {
  __shared__ double red[16][65];
  __shared__ double lds[2 * 17];
  if (done && *done != 0.0) return;
  if (k >= 0 && blockIdx.x == 0 && threadIdx.x < ACC_STRIDE) acc_set(d, k + 1)[threadIdx.x] = 0;
  const int lane = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  double* part = d.mv_part;
  double s = 0;
  if (e < d.nA) {
    if (d.det) {  // the deterministic product wrote every entry of row 0
      if (sl == 0) {
        s = part[e];
        if (!d.mv_lds) part[e] = 0;  // the atomic product accumulates into a zeroed row
      }
    } else if (d.mv_lds) {
      for (int w = sl; w < d.n_mv_wg; w += 16) s += part[(int64_t)w * d.nA + e];
    } else if (sl == 0) {
      s = part[e];
      part[e] = 0;
    }
  }
  red[sl][lane] = s;
  __syncthreads();
  double dot[1] = {0};
  if (sl == 0 && e < d.nA) {
    double t = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) t += red[j][lane];
    const double qv = t + lam * d.DA[e] * xin[e] + (d.n_rel ? d.rel_y[e] : 0.0);
    y[e] = qv;
    dot[0] = xin[e] * qv;
  }
  if (k < 0) return;
  double* const dst[1] = {acc_set(d, k) + ACC_PQ};
  block_atomic_add<1>(d, dot, lds, dst);
}

// alpha = rz / pq; x += alpha p, r -= alpha q; r.r (and Z^T r) -> set k   (one thread per entry)
template <bool COARSE> __global__ __launch_bounds__(256) void k_pcg_xr(Dev d, int k) {
  constexpr int NV = COARSE ? 1 + COARSE_K : 1;
  __shared__ double lds[5 * NV];
  if (d.scal[SC_DONE] != 0.0) return;
  const double pq = acc_set(d, k)[ACC_PQ];
  if (!(pq > 0.0) || !isfinite(pq)) {  // breakdown: keep x, stop
    if (blockIdx.x == 0 && threadIdx.x == 0) d.scal[SC_BREAK] = 1.0;
    return;
  }
  const double alpha = d.scal[SC_RZ] / pq;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  double v[NV];
#pragma unroll
  for (int a = 0; a < NV; ++a) v[a] = 0;
  if (e < d.nA) {
    d.x[e] += alpha * d.p[e];
    const double re = d.r[e] - alpha * d.q[e];
    d.r[e] = re;
    v[0] = re * re;
    if constexpr (COARSE) {
      for (int a = 0; a < d.coarse_k; ++a) v[1 + a] = d.Zc[(int64_t)a * d.nA + e] * re;
    }
  }
  double* A = acc_set(d, k);
  double* o = block_sum_arr<double, NV>(v, lds);
  if (threadIdx.x < NV) acc_add(d, threadIdx.x == 0 ? A + ACC_RR : A + ACC_ZR + threadIdx.x - 1, o[threadIdx.x]);
}

// z = M r (block diagonal); r.z -> set k; with the coarse space also (S Z)^T M r
// (the coarse part of z is added by k_pcg_p)   (one thread per entry)
template <int CD, bool COARSE> __global__ __launch_bounds__(256) void k_pcg_z(Dev d, int k) {
  constexpr int NV = COARSE ? 1 + COARSE_K : 1;
  __shared__ double lds[5 * NV];
  if (d.scal[SC_DONE] != 0.0 || d.scal[SC_BREAK] != 0.0) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  double v[NV];
#pragma unroll
  for (int a = 0; a < NV; ++a) v[a] = 0;
  if (e < d.nA) {
    int o, n;
    const double* M;
    entry_block<CD>(d, e, o, n, M);
    const int row = e - o;
    double t = 0;
    for (int c = 0; c < n; ++c) t += M[row * n + c] * d.r[o + c];
    d.z[e] = t;
    v[0] = d.r[e] * t;
    if constexpr (COARSE) {
      for (int a = 0; a < d.coarse_k; ++a) v[1 + a] = d.SZc[(int64_t)a * d.nA + e] * t;
    }
  }
  double* A = acc_set(d, k);
  double* o = block_sum_arr<double, NV>(v, lds);
  if (threadIdx.x < NV) acc_add(d, threadIdx.x == 0 ? A + ACC_RZ : A + ACC_W + threadIdx.x - 1, o[threadIdx.x]);
}

// beta = rz_k / rz_(k-1); p = z + beta p (z completed with the coarse term);
// workgroup 0 updates the scalars and the stopping test
template <typename T, bool COARSE> __global__ __launch_bounds__(256) void k_pcg_p(Dev d, int k) {
  __shared__ double ys[COARSE_K];
  __shared__ double rzs[2];
  if (d.scal[SC_DONE] != 0.0) return;
  const double* A = acc_set(d, k);
  if (d.scal[SC_BREAK] != 0.0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) d.scal[SC_DONE] = 1.0;
    return;
  }
  const double rr = A[ACC_RR];
  double rz = A[ACC_RZ];
  double rz_prev = acc_set(d, k + 2)[ACC_RZ];  // set (k - 1) mod 3
  const bool on = COARSE && d.scal[SC_COARSE] != 0.0;
  if (on) {
    // y = E^-1 (Z^T r - (S Z)^T M r) for this and the previous iteration, once per workgroup
    const int K = d.coarse_k;
    const double* Ap = acc_set(d, k + 2);
    static_assert(COARSE_K <= 16, "one 16-lane group per set");
    if (threadIdx.x < 32) {  // lanes 0-15: this iteration, 16-31: the previous one
      const int set = threadIdx.x >> 4, c = threadIdx.x & 15;
      const double* S = set == 0 ? A : Ap;
      double y = 0;
      if (c < K)
        for (int b = 0; b < K; ++b) y += d.Einv[c * COARSE_K + b] * (S[ACC_ZR + b] - S[ACC_W + b]);
      // r.z = r.(M r) + (Z^T r) . y
      double part = c < K ? S[ACC_ZR + c] * y : 0.0;
      for (int o = 8; o > 0; o >>= 1) part += __shfl_xor(part, o, 16);
      if (set == 0 && c < COARSE_K) ys[c] = y;
      if (c == 0) rzs[set] = part;
    }
    __syncthreads();
    rz += rzs[0];
    rz_prev += rzs[1];
  }
  const double beta = rz / rz_prev;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < d.nA) {
    double z = d.z[e];
    if (on)
      for (int c = 0; c < d.coarse_k; ++c) z += d.Zc[(int64_t)c * d.nA + e] * ys[c];
    const double pk = z + beta * d.p[e];
    d.p[e] = pk;
    ((T*)d.xT)[e] = (T)pk;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double iter = d.scal[SC_ITER] + 1.0;
    d.scal[SC_ITER] = iter;
    d.scal[SC_RR] = rr;
    d.scal[SC_RZ] = rz;
    d.scal[SC_PQ] = A[ACC_PQ];
    d.scal[SC_BETA] = beta;
    if (rr <= d.scal[SC_TOL2] || iter >= d.scal[SC_MAXIT] || !isfinite(rr)) d.scal[SC_DONE] = 1.0;
  }
}

// deterministic mode: sum the per-workgroup partials that a kernel of nwg workgroups just
// wrote for accumulator slots [lo, lo + n) and [lo2, lo2 + n2)
static void det_sum(const Dev& d, int lo, int n, int lo2, int n2, unsigned nwg, hipStream_t s) {
  if (d.det) k_det_sum<<<1, 64, 0, s>>>(d, lo, n, lo2, n2, (int)nwg);
}

static int acc_slot(int iter, int which) { return SC_ACC + ACC_STRIDE * (iter % 3) + which; }

// Every solve starts with the coarse-capable kernels, whose coarse terms are off unless a
// coarse space is active: block-Jacobi and a two-level solve whose coarse matrix turned
// out singular then run exactly the same arithmetic.
void launch_pcg_init(const Dev& d, double tol, int max_iters, hipStream_t s) {
  k_pcg_reset<<<1, 1, 0, s>>>(d, tol, max_iters);
  const unsigned gz = std::min(64u, nblk(d.nA, 256)), g = nblk(d.nA, 256);
  if (d.coarse_k > 0) {
    k_coarse_ztb<<<gz, 256, 0, s>>>(d);
    det_sum(d, SC_COUNT, COARSE_K, 0, 0, gz, s);
  }
  if (d.CD == 9) k_pcg_init_coarse<9><<<g, 256, 0, s>>>(d);
  else k_pcg_init_coarse<6><<<g, 256, 0, s>>>(d);
  det_sum(d, acc_slot(2, ACC_RZ), ACC_STRIDE - ACC_RZ, SC_BB, 1, g, s);
  if (d.fp64) k_pcg_init_coarse2<double><<<g, 256, 0, s>>>(d);
  else k_pcg_init_coarse2<float><<<g, 256, 0, s>>>(d);
  k_pcg_start<<<1, 1, 0, s>>>(d);
}

void launch_pcg_product(const Dev& d, hipStream_t s) { BA_DISPATCH_T_CD(d, run_matvec<T, CD>(d, d.scal + SC_DONE, s)); }

void launch_pcg_update(const Dev& d, double lambda, int iter, hipStream_t s) {
  const unsigned gq = nblk(d.nA, 64), g = nblk(d.nA, 256);
  const int kc = d.coarse_k > 0 ? COARSE_K : 0;
  BA_DISPATCH_T_CD(d, {
    k_pcg_q<T><<<gq, 1024, 0, s>>>(d, d.scal + SC_DONE, d.p, d.q, lambda, iter);
    det_sum(d, acc_slot(iter, ACC_PQ), 1, 0, 0, gq, s);
    if (d.coarse_k > 0) k_pcg_xr<true><<<g, 256, 0, s>>>(d, iter);
    else k_pcg_xr<false><<<g, 256, 0, s>>>(d, iter);
    det_sum(d, acc_slot(iter, ACC_RR), 1, acc_slot(iter, ACC_ZR), kc, g, s);
    if (d.coarse_k > 0) k_pcg_z<CD, true><<<g, 256, 0, s>>>(d, iter);
    else k_pcg_z<CD, false><<<g, 256, 0, s>>>(d, iter);
    det_sum(d, acc_slot(iter, ACC_RZ), 1, acc_slot(iter, ACC_W), kc, g, s);
    if (d.coarse_k > 0) k_pcg_p<T, true><<<g, 256, 0, s>>>(d, iter);
    else k_pcg_p<T, false><<<g, 256, 0, s>>>(d, iter);
  });
}

void launch_schur_matvec(const Dev& d, const double* xin, double* yout, double lambda, hipStream_t s) {
  BA_DISPATCH_T_CD(d, {
    k_to_T<T><<<nblk(d.nA, 256), 256, 0, s>>>(xin, d.xT, d.nA);
    run_matvec<T, CD>(d, nullptr, s);
    k_pcg_q<T><<<nblk(d.nA, 64), 1024, 0, s>>>(d, nullptr, xin, yout, lambda, -1);
  });
}

__global__ void k_unit_vector(double* v, int n, int c) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) v[e] = e == c ? 1.0 : 0.0;
}

void launch_dense_schur_columns(const Dev& d, double lambda, int c0, int ncols, double* S, hipStream_t s) {
  for (int c = 0; c < ncols; ++c) {
    k_unit_vector<<<std::min(64u, nblk(d.nA, 256)), 256, 0, s>>>(d.z, d.nA, c0 + c);
    launch_schur_matvec(d, d.z, S + (int64_t)c * d.nA, lambda, s);
  }
}

void launch_dense_schur(const Dev& d, double lambda, double* S, hipStream_t s) {
  launch_dense_schur_columns(d, lambda, 0, d.nA, S, s);
}

// E[a][b] = Z_a . (S Z)_b for the active columns, one workgroup per entry
__global__ __launch_bounds__(256) void k_coarse_e(Dev d, double* E) {
  __shared__ double lds[5];
  const int a = blockIdx.x / COARSE_K, b = blockIdx.x % COARSE_K;
  double v[1] = {0};
  if (a < d.coarse_k && b < d.coarse_k)
    for (int e = threadIdx.x; e < d.nA; e += blockDim.x) v[0] += d.Zc[(int64_t)a * d.nA + e] * d.SZc[(int64_t)b * d.nA + e];
  double* o = block_sum_arr<double, 1>(v, lds);
  if (threadIdx.x == 0) E[blockIdx.x] = o[0];
}

// Einv = E^-1 of the symmetrised E (active K x K part) by Gauss-Jordan elimination
// without pivoting (E is symmetric positive definite: every pivot is a positive
// Schur complement); SC_COARSE = 0 when a pivot is not positive or the inverse is
// not finite.  One workgroup, one thread per entry of [E | I].
__global__ __launch_bounds__(512) void k_coarse_inv(Dev d, const double* E) {
  constexpr int Kc = COARSE_K;
  __shared__ double A[Kc][2 * Kc];
  __shared__ int bad;
  const int K = d.coarse_k, t = threadIdx.x;
  const int r = t / (2 * Kc), c = t % (2 * Kc);
  const bool mine = r < K && (c < K || (c >= Kc && c < Kc + K));
  if (t == 0) bad = K <= 0 ? 1 : 0;
  if (t < Kc * 2 * Kc) A[r][c] = !mine ? 0.0 : c < K ? 0.5 * (E[r * Kc + c] + E[c * Kc + r]) : (c - Kc == r ? 1.0 : 0.0);
  __syncthreads();
  for (int p = 0; p < K; ++p) {
    const double piv = A[p][p];
    const double f = t < Kc * 2 * Kc ? A[r][p] : 0.0;
    const double prow = t < Kc * 2 * Kc ? A[p][c] : 0.0;
    __syncthreads();
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (t == 0) bad = 1;
    } else if (mine) {
      A[r][c] = r == p ? prow / piv : A[r][c] - f * prow / piv;
    }
    __syncthreads();
  }
  const bool ok = bad == 0;
  if (t < Kc * Kc) {
    const int i = t / Kc, j = t % Kc;
    double v = 0.0;
    if (ok && i < K && j < K) v = 0.5 * (A[i][Kc + j] + A[j][Kc + i]);
    d.Einv[t] = isfinite(v) ? v : 0.0;
    if (!isfinite(v)) atomicAdd(&bad, 1);
  }
  __syncthreads();
  if (t == 0) d.scal[SC_COARSE] = bad == 0 ? 1.0 : 0.0;
}

// similarity-gauge columns (rotation x, y, z; translation x, y, z; scale) of every
// camera / plane / VP block, from the current FP64 parameters (one thread per block)
__global__ void k_gauge_basis(Dev d) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= d.nc + d.ng + d.nv) return;
  double g[9][COARSE_GAUGE];
  int o, n;
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < COARSE_GAUGE; ++c) g[r][c] = 0.0;
  if (b < d.nc) {
    const double* cam = d.cam64 + (int64_t)CAM_STRIDE * b;  // R row-major, t
    const double* t = cam + 9;
    o = d.CD * b;
    n = d.CD;
    for (int k = 0; k < 3; ++k) {
      const double Rk[3] = {cam[k], cam[3 + k], cam[6 + k]};  // R e_k
      // rotation: dtheta = -R e_k, dt = (R e_k) x t; translation: dt = -R e_k
      g[0][k] = -Rk[0]; g[1][k] = -Rk[1]; g[2][k] = -Rk[2];
      g[3][k] = Rk[1] * t[2] - Rk[2] * t[1];
      g[4][k] = Rk[2] * t[0] - Rk[0] * t[2];
      g[5][k] = Rk[0] * t[1] - Rk[1] * t[0];
      g[3][3 + k] = -Rk[0]; g[4][3 + k] = -Rk[1]; g[5][3 + k] = -Rk[2];
    }
    g[3][6] = t[0]; g[4][6] = t[1]; g[5][6] = t[2];
  } else if (b < d.nc + d.ng) {
    const int q = b - d.nc;
    const double* pl = d.pl64 + (int64_t)PL_STRIDE * q;  // n, w, b1, b2
    o = d.offPl + 3 * q;
    n = 3;
    for (int k = 0; k < 3; ++k) {
      double en[3] = {0, 0, 0};  // e_k x n
      en[(k + 1) % 3] = -pl[(k + 2) % 3];
      en[(k + 2) % 3] = pl[(k + 1) % 3];
      g[0][k] = pl[4] * en[0] + pl[5] * en[1] + pl[6] * en[2];
      g[1][k] = pl[7] * en[0] + pl[8] * en[1] + pl[9] * en[2];
      g[2][3 + k] = -pl[k];
    }
    g[2][6] = pl[3];
  } else {
    const int q = b - d.nc - d.ng;
    const double* vp = d.vp64 + (int64_t)VP_STRIDE * q;  // v, pad, b1, b2
    o = d.offVp + 2 * q;
    n = 2;
    for (int k = 0; k < 3; ++k) {
      double ev[3] = {0, 0, 0};  // e_k x v
      ev[(k + 1) % 3] = -vp[(k + 2) % 3];
      ev[(k + 2) % 3] = vp[(k + 1) % 3];
      g[0][k] = vp[4] * ev[0] + vp[5] * ev[1] + vp[6] * ev[2];
      g[1][k] = vp[7] * ev[0] + vp[8] * ev[1] + vp[9] * ev[2];
    }
  }
  for (int c = 0; c < COARSE_GAUGE; ++c)
    for (int r = 0; r < n; ++r) d.Zc[(int64_t)c * d.nA + o + r] = g[r][c];
}

void launch_gauge_basis(const Dev& d, hipStream_t s) {
  const int nb = d.nc + d.ng + d.nv;
  if (nb > 0) k_gauge_basis<<<nblk(nb, 64), 64, 0, s>>>(d);
  launch_shape_gauge(d, s);
}

// ---- S Z for the coarse columns ---------------------------------------------
// S x = sum_r J_a,r^T (J_a,r x - J_f,r s_f) + lambda D_a x, s_f = V_f^-1 sum_{r in f} J_f,r^T J_a,r x
// Z rows and s_f are stored in panels of SZ_COLS columns (row-major in a panel): the gauge
// columns in panel 0, the network's in panel 1.  s_f of a panel: a feature sweep over the
// product's wavefront tiles, or, for the gauge panel when no VP 3-vector record exists,
// the closed form of k_sz_gauge_feat.  Camera / group sweeps, all columns in one launch: a
// workgroup per camera / group owns that block of the output (no atomics), and each of its
// records is taken by SZ_LANES lanes per panel.
// Two lanes of four columns each balance the slot loads, repeated on every lane of a
// record, against the registers of the FP64 sums (1M-point scene, 15 columns: 1, 2, 4, 8
// lanes per panel gave 4.9, 4.2, 4.3, 5.1 ms for the preconditioner set-up).
constexpr int SZ_LANES = 2;
struct SzPanels {
  int64_t z, p, l;  // panel strides of Z rows, point s_f, line s_f
};
__host__ __device__ inline SzPanels sz_panels(const Dev& d) { return {(int64_t)d.nA * SZ_COLS, (int64_t)d.np * 3 * SZ_COLS, (int64_t)d.nl * 4 * SZ_COLS}; }

// coarse column held by slot s of panel pn: panel 0 the gauge columns, panel 1 the
// network's; -1 for an unused slot
static_assert(SZ_PANELS == 2 && COARSE_GAUGE <= SZ_COLS && COARSE_NET <= SZ_COLS, "gauge panel, network panel");
__host__ __device__ inline int sz_col(int pn, int s) { return pn == 0 ? (s < COARSE_GAUGE ? s : -1) : COARSE_GAUGE + s; }

// Z rows in T: Zr[pn][e][s] = Z[sz_col(pn, s)][e], zero in unused slots and, with
// gauge_zero, in the gauge panel (its s_f then come in closed form, see k_sz_gauge_feat)
template <typename T> __global__ void k_sz_rows(Dev d, T* Zr, int gauge_zero) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t panel = (int64_t)d.nA * SZ_COLS;
  if (t >= panel * SZ_PANELS) return;
  const int pn = (int)(t / panel), e = (int)((t % panel) / SZ_COLS);
  const int c = sz_col(pn, (int)(t % SZ_COLS));
  Zr[t] = c < 0 || c >= d.coarse_k || (pn == 0 && gauge_zero) ? (T)0 : (T)d.Zc[(int64_t)c * d.nA + e];
}

// The gauge panel in closed form.  With z = (z_a, z_f) the first-order motion of every
// parameter under a world rotation, translation or scale (z_a: the gauge columns of Z),
// J z = 0 for every family but the VP 3-vector, whose value turns with the world: then
// W^T z_a = -V z_f and U z_a = -W z_f, so
//   S z_a = lambda D_a z_a - lambda W (V + lambda D_f)^-1 D_f z_f.
// The camera / group sweeps form exactly this when the gauge panel's Z rows are zero and
// its s_f = lambda (V + lambda D_f)^-1 D_f z_f, which this kernel writes (one thread per
// point, then per line), reading no record.  Points move additively: e_k x X, e_k, X.  A
// line (U, w1, w2) moves by dtheta = U^T e_k under rotation k, by dtheta =
// (-w1 (u2 . e_k) / w2, 0, 0) and dphi = w1^2 (u3 . e_k) under translation k, and by
// dphi = w1 w2 under the scale.
template <typename T, int NF>
__device__ __forceinline__ void sz_gauge_solve(const Dev& d, int f, const double (&z)[NF][COARSE_GAUGE], double lam, T* sf) {
  const double* D = (NF == 3 ? d.Dp : d.Dl) + (int64_t)NF * f;
  T o[NF * SZ_COLS];  // the feature's rows of the panel, stored in one vector write
#pragma unroll
  for (int k = 0; k < NF * SZ_COLS; ++k) o[k] = (T)0;
#pragma unroll
  for (int c = 0; c < COARSE_GAUGE; ++c) {
    T q[NF], y[NF];
#pragma unroll
    for (int a = 0; a < NF; ++a) q[a] = (T)(D[a] * z[a][c]);
    apply_vinv<T, NF>(d, f, q, y);
#pragma unroll
    for (int a = 0; a < NF; ++a) o[a * SZ_COLS + c] = (T)(lam * (double)y[a]);
  }
  store_vec(sf + (int64_t)f * NF * SZ_COLS, o);
}

template <typename T> __global__ void k_sz_gauge_feat(Dev d, T* sfp, T* sfl, double lam) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < d.np) {
    const double* X = d.pt64 + (int64_t)PT_STRIDE * f;
    double z[3][COARSE_GAUGE];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < COARSE_GAUGE; ++c) z[a][c] = 0.0;
    z[1][0] = -X[2]; z[2][0] = X[1];  // e_0 x X
    z[0][1] = X[2]; z[2][1] = -X[0];  // e_1 x X
    z[0][2] = -X[1]; z[1][2] = X[0];  // e_2 x X
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      z[a][3 + a] = 1.0;
      z[a][6] = X[a];
    }
    sz_gauge_solve<T, 3>(d, f, z, lam, sfp);
  } else if (f < d.np + d.nl) {
    const int j = f - d.np;
    const double* L = d.ln64 + (int64_t)LN_STRIDE * j;  // u1, u2, u3, w1, w2
    const double w1 = L[9], w2 = L[10];
    double z[4][COARSE_GAUGE];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < COARSE_GAUGE; ++c) z[a][c] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      z[0][k] = L[k];
      z[1][k] = L[3 + k];
      z[2][k] = L[6 + k];
      z[0][3 + k] = w2 != 0.0 ? -w1 * L[3 + k] / w2 : 0.0;
      z[3][3 + k] = w1 * w1 * L[6 + k];
    }
    z[3][6] = w1 * w2;
    sz_gauge_solve<T, 4>(d, j, z, lam, sfl);
  }
}

// t[row][c] = (J_a Z_r)[row][c] for one record (Zr: one panel)
template <int FAM, typename T, int CD>
__device__ __forceinline__ void sz_record_t(const Dev& d, int64_t i, const T* Zr, const T (&v)[Slot<FAM, CD>::STRIDE],
                                            T (&t)[4][SZ_COLS]) {
  using SL = Slot<FAM, CD>;
  using F = Fam<FAM, CD>;
#pragma unroll
  for (int row = 0; row < 4; ++row)
#pragma unroll
    for (int c = 0; c < SZ_COLS; ++c) t[row][c] = 0;
  if constexpr (SL::NC > 0) {
    const T* z = Zr + (int64_t)CD * d.fcam[FAM][i] * SZ_COLS;
#pragma unroll
    for (int k = 0; k < SL::NC; ++k)
#pragma unroll
      for (int c = 0; c < SZ_COLS; ++c) {
        const T zk = z[k * SZ_COLS + c];
#pragma unroll
        for (int row = 0; row < SL::ROWS; ++row) t[row][c] += v[SL::OC + row * SL::NC + k] * zk;
      }
  }
  if constexpr (SL::NG > 0) {
    const T* z = Zr + (int64_t)a_grp(d, F::GT, d.fgrp[FAM][i]) * SZ_COLS;
#pragma unroll
    for (int k = 0; k < SL::NG; ++k)
#pragma unroll
      for (int c = 0; c < SZ_COLS; ++c) {
        const T zk = z[k * SZ_COLS + c];
#pragma unroll
        for (int row = 0; row < SL::ROWS; ++row) t[row][c] += v[SL::OG + row * SL::NG + k] * zk;
      }
  }
}


// s_f = (V_f + lambda D_f)^-1 q for the SZ_COLS columns of one feature, stored to its
// contiguous NF x SZ_COLS block of sf: the feature's FP32 inverse is read once (not per
// column after the column's stores, which may alias it); a flagged block takes its FP64
// inverse column by column
template <typename T, int NF, int QF>
__device__ __forceinline__ void sz_solve_store(const Dev& d, int f, const T (&q)[QF][SZ_COLS], T* sf) {
  constexpr int NS = NF * (NF + 1) / 2;
  T out[NF][SZ_COLS];
  if ((NF == 3 ? d.flp : d.fll)[f]) {
    for (int c = 0; c < SZ_COLS; ++c) {
      T qc[NF], sc[NF];
#pragma unroll
      for (int a = 0; a < NF; ++a) qc[a] = q[a][c];
      apply_vinv<T, NF>(d, f, qc, sc);
#pragma unroll
      for (int a = 0; a < NF; ++a) out[a][c] = sc[a];
    }
  } else {
    const T* M = (const T*)(NF == 3 ? d.Vip : d.Vil) + (int64_t)NS * f;
    T m[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) m[k] = M[k];
#pragma unroll
    for (int c = 0; c < SZ_COLS; ++c)
#pragma unroll
      for (int a = 0; a < NF; ++a) {
        T t = 0;
#pragma unroll
        for (int b = 0; b < NF; ++b) t += m[sym<NF>(a, b)] * q[b][c];
        out[a][c] = t;
      }
  }
  T* o = sf + (int64_t)f * NF * SZ_COLS;
#pragma unroll
  for (int a = 0; a < NF; ++a)
#pragma unroll
    for (int c = 0; c < SZ_COLS; ++c) o[a * SZ_COLS + c] = out[a][c];
}

// one record's J_f^T J_a Z (SZ_COLS columns of one panel) added to q: the slot loaded
// whole, or a row at a time for the surface-group families
template <int FAM, typename T, int CD, int NF>
__device__ __forceinline__ void sz_rec_q(const Dev& d, int64_t i, const T* Zr, T (&q)[NF][SZ_COLS]) {
  using SL = Slot<FAM, CD>;
  if constexpr (Fam<FAM, CD>::GT == 3) {
    const T* sl = (const T*)d.frec[FAM] + i * SL::STRIDE;
    const T* zc = Zr + (int64_t)CD * d.fcam[FAM][i] * SZ_COLS;
    const T* zg = Zr + (int64_t)a_grp(d, 3, d.fgrp[FAM][i]) * SZ_COLS;
#pragma unroll 1
    for (int row = 0; row < SL::ROWS; ++row) {
      T t[SZ_COLS];
#pragma unroll
      for (int c = 0; c < SZ_COLS; ++c) t[c] = 0;
#pragma unroll
      for (int k = 0; k < SL::NC; ++k) {
        const T j = sl[SL::OC + row * SL::NC + k];
#pragma unroll
        for (int c = 0; c < SZ_COLS; ++c) t[c] += j * zc[k * SZ_COLS + c];
      }
#pragma unroll
      for (int k = 0; k < SL::NG; ++k) {
        const T j = sl[SL::OG + row * SL::NG + k];
#pragma unroll
        for (int c = 0; c < SZ_COLS; ++c) t[c] += j * zg[k * SZ_COLS + c];
      }
#pragma unroll
      for (int a = 0; a < NF; ++a) {
        const T j = sl[SL::OF + row * NF + a];
#pragma unroll
        for (int c = 0; c < SZ_COLS; ++c) q[a][c] += j * t[c];
      }
    }
  } else {
    T v[SL::STRIDE];
    load_vec((const T*)d.frec[FAM] + i * SL::STRIDE, v);
    T t[4][SZ_COLS];
    sz_record_t<FAM, T, CD>(d, i, Zr, v, t);
#pragma unroll
    for (int a = 0; a < NF; ++a)
#pragma unroll
      for (int c = 0; c < SZ_COLS; ++c) {
        T acc = 0;
#pragma unroll
        for (int row = 0; row < SL::ROWS; ++row) acc += v[SL::OF + row * NF + a] * t[row][c];
        q[a][c] += acc;
      }
  }
}

template <int FAM, typename T, int CD, int NF>
__device__ __forceinline__ void sz_wave_family(const Dev& d, int f, const T* Zr, int& j0, int lane, T (&q)[NF][SZ_COLS]) {
  if (!d.fn[FAM]) return;
  const int64_t b = d.foff[FAM][f];
  const int n = (int)(d.foff[FAM][f + 1] - b);
  // record r of the family is on lane (j0 + r) mod 64
  for (int r = (lane - j0 % 64 + 64) % 64; r < n; r += 64) sz_rec_q<FAM, T, CD, NF>(d, b + r, Zr, q);
  j0 += n;
}

// s_f of one feature larger than a tile (or a line on a shape), one wavefront: its
// records over the lanes, q summed across the wavefront, solved and stored by lane 0
// (Zr, sf: one panel). Every lane calls this with the same f, and all are active.
template <typename T, int CD, int NF> __device__ __forceinline__ void sz_feature_wave(const Dev& d, int f, const T* Zr, T* sf, int lane) {
  T q[NF][SZ_COLS];
#pragma unroll
  for (int a = 0; a < NF; ++a)
#pragma unroll
    for (int c = 0; c < SZ_COLS; ++c) q[a][c] = 0;
  int j0 = 0;
  if constexpr (NF == 3) {
    sz_wave_family<1, T, CD, 3>(d, f, Zr, j0, lane, q);
    sz_wave_family<3, T, CD, 3>(d, f, Zr, j0, lane, q);
    sz_wave_family<6, T, CD, 3>(d, f, Zr, j0, lane, q);
    sz_wave_family<8, T, CD, 3>(d, f, Zr, j0, lane, q);
    sz_wave_family<9, T, CD, 3>(d, f, Zr, j0, lane, q);
  } else {
    sz_wave_family<2, T, CD, 4>(d, f, Zr, j0, lane, q);
    sz_wave_family<4, T, CD, 4>(d, f, Zr, j0, lane, q);
    sz_wave_family<5, T, CD, 4>(d, f, Zr, j0, lane, q);
    sz_wave_family<7, T, CD, 4>(d, f, Zr, j0, lane, q);
    sz_wave_family<10, T, CD, 4>(d, f, Zr, j0, lane, q);
  }
#pragma unroll
  for (int a = 0; a < NF; ++a)
#pragma unroll
    for (int c = 0; c < SZ_COLS; ++c) q[a][c] = wave_sum(q[a][c]);
  if (lane == 0) sz_solve_store<T, NF>(d, f, q, sf);
}


// features larger than a product tile (and lines on a shape), one wavefront per listed
// feature
template <typename T, int CD, int NF> __global__ __launch_bounds__(256) void k_sz_feat_big(Dev d, const T* Zr, T* sf, const int32_t* list, int n) {
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int k = blockIdx.x * nw + (threadIdx.x >> 6); k < n; k += gridDim.x * nw) sz_feature_wave<T, CD, NF>(d, list[k], Zr, sf, lane);
}

// q[a][c] = sum over rows of J_f[row][a] (J_a Z_r)[row][c] for one record
template <int FAM, typename T, int CD>
__device__ __forceinline__ void sz_wave_q(const Dev& d, int64_t i, int cam, int grp, const T* Zr, T (&q)[4][SZ_COLS]) {
  using SL = Slot<FAM, CD>;
  using F = Fam<FAM, CD>;
  T v[SL::STRIDE];
  load_vec(((const T*)d.frec[FAM]) + i * SL::STRIDE, v);
  T t[4][SZ_COLS];
#pragma unroll
  for (int row = 0; row < 4; ++row)
#pragma unroll
    for (int c = 0; c < SZ_COLS; ++c) t[row][c] = 0;
  if constexpr (SL::NC > 0) {
    const T* z = Zr + (int64_t)CD * cam * SZ_COLS;
#pragma unroll
    for (int k = 0; k < SL::NC; ++k)
#pragma unroll
      for (int c = 0; c < SZ_COLS; ++c) {
        const T zk = z[k * SZ_COLS + c];
#pragma unroll
        for (int row = 0; row < SL::ROWS; ++row) t[row][c] += v[SL::OC + row * SL::NC + k] * zk;
      }
  }
  if constexpr (SL::NG > 0) {
    const T* z = Zr + (int64_t)a_grp(d, F::GT, grp) * SZ_COLS;
#pragma unroll
    for (int k = 0; k < SL::NG; ++k)
#pragma unroll
      for (int c = 0; c < SZ_COLS; ++c) {
        const T zk = z[k * SZ_COLS + c];
#pragma unroll
        for (int row = 0; row < SL::ROWS; ++row) t[row][c] += v[SL::OG + row * SL::NG + k] * zk;
      }
  }
#pragma unroll
  for (int a = 0; a < SL::NF; ++a)
#pragma unroll
    for (int c = 0; c < SZ_COLS; ++c) {
      T acc = 0;
#pragma unroll
      for (int row = 0; row < SL::ROWS; ++row) acc += v[SL::OF + row * SL::NF + a] * t[row][c];
      q[a][c] = acc;
    }
}

// s_f of every feature over the product's wavefront tiles: one record per lane,
// the feature sums of J_f^T J_a Z by a segmented scan across the wavefront, the
// solve on the feature's last lane (Zr, sfp, sfl: one panel)
template <typename T, int CD> __global__ __launch_bounds__(256) void k_sz_feat_wave(Dev d, const T* Zr, T* sfp, T* sfl) {
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int tile = blockIdx.x * nw + (threadIdx.x >> 6); tile < d.n_tiles; tile += gridDim.x * nw) {
    const int4 tl = d.tiles[tile];
    const int fb = tl.z;
    const bool active = lane < tl.y;
    const bool ptile = tile < d.n_ptiles;
    int4 w4 = make_int4(0, 0, 0, -1);
    if (active) w4 = d.wrec[tl.x + lane];
    const int fam = (int)((uint32_t)w4.x >> 28), lf = w4.w;
    const int64_t i = (int64_t)((uint32_t)w4.x & 0x0fffffffu);
    T q[4][SZ_COLS];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < SZ_COLS; ++c) q[a][c] = 0;
    if (active) {
      switch (fam) {
        case 1: sz_wave_q<1, T, CD>(d, i, w4.y, w4.z, Zr, q); break;
        case 2: sz_wave_q<2, T, CD>(d, i, w4.y, w4.z, Zr, q); break;
        case 3: sz_wave_q<3, T, CD>(d, i, w4.y, w4.z, Zr, q); break;
        case 4: sz_wave_q<4, T, CD>(d, i, w4.y, w4.z, Zr, q); break;
        case 5: sz_wave_q<5, T, CD>(d, i, w4.y, w4.z, Zr, q); break;
        case 6: sz_wave_q<6, T, CD>(d, i, w4.y, w4.z, Zr, q); break;
        case 7: sz_wave_q<7, T, CD>(d, i, w4.y, w4.z, Zr, q); break;
        case 8: sz_wave_q<8, T, CD>(d, i, w4.y, w4.z, Zr, q); break;
        case 9: sz_wave_q<9, T, CD>(d, i, w4.y, w4.z, Zr, q); break;
      }
    }
    const int prev = __shfl_up(lf, 1, 64);
    const unsigned long long heads = __ballot(lf >= 0 && (lane == 0 || prev != lf));
    const int start = lf >= 0 ? 63 - __builtin_clzll(heads & ((2ull << lane) - 1ull)) : lane;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const bool take = lane - off >= start;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (a == 3 && ptile) continue;
#pragma unroll
        for (int c = 0; c < SZ_COLS; ++c) {
          const T o = __shfl_up(q[a][c], off, 64);
          if (take) q[a][c] += o;
        }
      }
    }
    const int next = __shfl_down(lf, 1, 64);
    if (lf >= 0 && (lane == 63 || next != lf)) {
      if (ptile) sz_solve_store<T, 3>(d, fb + lf, q, sfp);
      else sz_solve_store<T, 4>(d, fb + lf, q, sfl);
    }
  }
}

// CPL consecutive columns of N rows of Z from row e0 (Zr: the panel, offset to the first
// of the columns)
template <int N, int CPL, typename T> __device__ __forceinline__ void z_cols(const T* Zr, int e0, T (&z)[N][CPL]) {
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int c = 0; c < CPL; ++c) z[k][c] = Zr[(int64_t)(e0 + k) * SZ_COLS + c];
}

// one record, CPL columns: u = J_a z - J_f s_f (s: the feature's s_f at the first column),
// then the camera (OUT 0) or group (OUT 1) rows of J^T u added to acc
template <int FAM, int OUT, typename T, int CD, int NO, int CPL>
__device__ __forceinline__ void sz_rec_cols(const T* slot, const T (&zc)[CD][CPL], const T (&zg)[3][CPL], const T* s,
                                            double (&acc)[NO][CPL], int ss = SZ_COLS) {
  using SL = Slot<FAM, CD>;
  static_assert(NO >= (OUT == 0 ? SL::NC : SL::NG), "output rows");
  T v[SL::STRIDE];
  load_vec(slot, v);
  T sf[SL::NF][CPL];
#pragma unroll
  for (int a = 0; a < SL::NF; ++a)
#pragma unroll
    for (int c = 0; c < CPL; ++c) sf[a][c] = s[a * ss + c];
  T u[SL::ROWS][CPL];
#pragma unroll
  for (int row = 0; row < SL::ROWS; ++row)
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      T t = 0;
#pragma unroll
      for (int k = 0; k < SL::NC; ++k) t += v[SL::OC + row * SL::NC + k] * zc[k][c];
#pragma unroll
      for (int k = 0; k < SL::NG; ++k) t += v[SL::OG + row * SL::NG + k] * zg[k][c];
#pragma unroll
      for (int a = 0; a < SL::NF; ++a) t -= v[SL::OF + row * SL::NF + a] * sf[a][c];
      u[row][c] = t;
    }
  constexpr int NK = OUT == 0 ? SL::NC : SL::NG, O = OUT == 0 ? SL::OC : SL::OG;
#pragma unroll
  for (int k = 0; k < NK; ++k)
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      T t = 0;
#pragma unroll
      for (int row = 0; row < SL::ROWS; ++row) t += v[O + row * NK + k] * u[row][c];
      acc[k][c] += (double)t;
    }
}

// sum of acc over the lanes of a 256-thread workgroup that hold the same columns (lane
// mod L, L lanes per record), then out(row, column, sum) on the first NO * L * CPL threads
template <int NO, int L, int CPL, typename Out>
__device__ __forceinline__ void sz_block_sum(double (&acc)[NO][CPL], double* lds, Out out) {
  constexpr int NCOL = L * CPL;
#pragma unroll
  for (int k = 0; k < NO; ++k)
#pragma unroll
    for (int c = 0; c < CPL; ++c)
#pragma unroll
      for (int o = L; o < 64; o <<= 1) acc[k][c] += __shfl_xor(acc[k][c], o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l < L)
#pragma unroll
    for (int k = 0; k < NO; ++k)
#pragma unroll
      for (int c = 0; c < CPL; ++c) lds[(w * NO + k) * NCOL + l * CPL + c] = acc[k][c];
  __syncthreads();
  for (int t = threadIdx.x; t < NO * NCOL; t += blockDim.x)
    out(t / NCOL, t % NCOL, lds[t] + lds[NO * NCOL + t] + lds[2 * NO * NCOL + t] + lds[3 * NO * NCOL + t]);
}

// output rows of one camera (workgroup of 256 per camera): S Z = sum over its records
// J_c^T u + lambda D Z.  L lanes per record, CPL columns per lane.
template <typename T, int CD, int L, int CPL>
__global__ __launch_bounds__(256) void k_sz_cam(Dev d, const T* Zr, const T* sfp, const T* sfl, double lam) {
  constexpr int R = 256 / L, NCOL = L * CPL;
  static_assert(SZ_COLS % CPL == 0, "a lane's columns lie in one panel");
  __shared__ double lds[4 * CD * NCOL];
  const int c = d.cam_order[blockIdx.x], col = (threadIdx.x % L) * CPL, rs = threadIdx.x / L;
  const SzPanels P = sz_panels(d);
  const int pn = col / SZ_COLS, pc = col % SZ_COLS;
  const T* zr = Zr + pn * P.z + pc;
  const T* sp = sfp + pn * P.p + pc;
  const T* sl = sfl + pn * P.l + pc;
  T zc[CD][CPL], z0[3][CPL];
  z_cols<CD, CPL>(zr, CD * c, zc);
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int q = 0; q < CPL; ++q) z0[k][q] = 0;
  double acc[CD][CPL];
#pragma unroll
  for (int k = 0; k < CD; ++k)
#pragma unroll
    for (int q = 0; q < CPL; ++q) acc[k][q] = 0;
  // observation slots and their aligned plane slots from the camera-major copies
  if (d.fn[1])
    for (int j = d.po_off[c] + rs; j < d.po_off[c + 1]; j += R) {
      const int f = d.cmfeat[1][j];
      sz_rec_cols<1, 0, T, CD>((const T*)d.cmrec[1] + (int64_t)j * Slot<1, CD>::STRIDE, zc, z0, sp + (int64_t)f * 3 * SZ_COLS, acc);
      const int k = d.cmal[1][j];
      if (k >= 0) {
        T zg[3][CPL];
        z_cols<3, CPL>(zr, a_grp(d, Fam<3, CD>::GT, d.cmgrp[3][k]), zg);
        sz_rec_cols<3, 0, T, CD>((const T*)d.cmrec[3] + (int64_t)k * Slot<3, CD>::STRIDE, zc, zg, sp + (int64_t)f * 3 * SZ_COLS, acc);
      }
    }
  // the camera's point-on-shape and line-on-cuboid records, in loops of their own
  if (d.shc_off[0])
    for (int j = d.shc_off[0][c] + rs; j < d.shc_off[0][c + 1]; j += R)
      sz_shape_rec<9, 0, T, CD, CPL>(d, d.shc_rec[0][j], zc, zr, sp + (int64_t)d.shc_feat[0][j] * 3 * SZ_COLS, acc);
  if (d.shc_off[1])
    for (int j = d.shc_off[1][c] + rs; j < d.shc_off[1][c + 1]; j += R)
      sz_shape_rec<10, 0, T, CD, CPL>(d, d.shc_rec[1][j], zc, zr, sl + (int64_t)d.shc_feat[1][j] * 4 * SZ_COLS, acc);
  if (d.fn[6])
    for (int j = d.px_off[c] + rs; j < d.px_off[c + 1]; j += R)
      for (int64_t i = d.px_start[j]; i < d.px_start[j] + d.px_cnt[j]; ++i)
        sz_rec_cols<6, 0, T, CD>((const T*)d.frec[6] + i * Slot<6, CD>::STRIDE, zc, z0, sp + (int64_t)d.ffeat[6][i] * 3 * SZ_COLS, acc);
  if (d.fn[2])
    for (int j = d.lo_off[c] + rs; j < d.lo_off[c + 1]; j += R) {
      const int f = d.cmfeat[2][j];
      sz_rec_cols<2, 0, T, CD>((const T*)d.cmrec[2] + (int64_t)j * Slot<2, CD>::STRIDE, zc, z0, sl + (int64_t)f * 4 * SZ_COLS, acc);
      const int k = d.cmal[2][j];
      if (k >= 0) {
        T zg[3][CPL];
        z_cols<3, CPL>(zr, a_grp(d, Fam<4, CD>::GT, d.cmgrp[4][k]), zg);
        sz_rec_cols<4, 0, T, CD>((const T*)d.cmrec[4] + (int64_t)k * Slot<4, CD>::STRIDE, zc, zg, sl + (int64_t)f * 4 * SZ_COLS, acc);
      }
    }
  if (d.fn[7])
    for (int j = d.lx_off[c] + rs; j < d.lx_off[c + 1]; j += R)
      for (int64_t i = d.lx_start[j]; i < d.lx_start[j] + d.lx_cnt[j]; ++i)
        sz_rec_cols<7, 0, T, CD>((const T*)d.frec[7] + i * Slot<7, CD>::STRIDE, zc, z0, sl + (int64_t)d.ffeat[7][i] * 4 * SZ_COLS, acc);
  sz_block_sum<CD, L, CPL>(acc, lds, [&](int row, int cc, double s) {
    const int col = sz_col(cc / SZ_COLS, cc % SZ_COLS);
    if (col < 0 || col >= d.coarse_k) return;
    const int e = CD * c + row;
    d.SZc[(int64_t)col * d.nA + e] = s + lam * d.DA[e] * d.Zc[(int64_t)col * d.nA + e];
  });
}

// output rows of one plane or VP (workgroup of 256 per group)
template <typename T, int CD, int L, int CPL>
__global__ __launch_bounds__(256) void k_sz_grp(Dev d, const T* Zr, const T* sfp, const T* sfl, double lam) {
  constexpr int R = 256 / L, NCOL = L * CPL;
  __shared__ double lds[4 * 3 * NCOL];
  const int col = (threadIdx.x % L) * CPL, rs = threadIdx.x / L;
  const SzPanels P = sz_panels(d);
  const int pn = col / SZ_COLS, pc = col % SZ_COLS;
  const T* zr = Zr + pn * P.z + pc;
  const T* sp = sfp + pn * P.p + pc;
  const T* sl = sfl + pn * P.l + pc;
  if ((int)blockIdx.x < d.ng) {
    const int g = blockIdx.x, e0 = a_grp(d, 1, g);
    T zg[3][CPL];
    z_cols<3, CPL>(zr, e0, zg);
    double acc[3][CPL];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int q = 0; q < CPL; ++q) acc[k][q] = 0;
    if (d.fn[3] || d.fn[8])
      for (int j = d.plp_off[g] + rs; j < d.plp_off[g + 1]; j += R) {
        const int f = d.plp[j];
        for (int64_t i = d.foff[3][f]; i < d.foff[3][f + 1]; ++i) {
          if (d.fgrp[3][i] != g) continue;
          T zc[CD][CPL];
          z_cols<CD, CPL>(zr, CD * d.fcam[3][i], zc);
          sz_rec_cols<3, 1, T, CD>((const T*)d.frec[3] + i * Slot<3, CD>::STRIDE, zc, zg, sp + (int64_t)f * 3 * SZ_COLS, acc);
        }
        for (int64_t i = d.foff[8][f]; i < d.foff[8][f + 1]; ++i) {
          if (d.fgrp[8][i] != g) continue;
          T zc[CD][CPL];
#pragma unroll
          for (int k = 0; k < CD; ++k)
#pragma unroll
            for (int q = 0; q < CPL; ++q) zc[k][q] = 0;
          sz_rec_cols<8, 1, T, CD>((const T*)d.frec[8] + i * Slot<8, CD>::STRIDE, zc, zg, sp + (int64_t)f * 3 * SZ_COLS, acc);
        }
      }
    if (d.fn[4])
      for (int j = d.pll_off[g] + rs; j < d.pll_off[g + 1]; j += R) {
        const int f = d.pll[j];
        for (int64_t i = d.foff[4][f]; i < d.foff[4][f + 1]; ++i) {
          T zc[CD][CPL];
          z_cols<CD, CPL>(zr, CD * d.fcam[4][i], zc);
          sz_rec_cols<4, 1, T, CD>((const T*)d.frec[4] + i * Slot<4, CD>::STRIDE, zc, zg, sl + (int64_t)f * 4 * SZ_COLS, acc);
        }
      }
    sz_block_sum<3, L, CPL>(acc, lds, [&](int row, int cc, double s) {
      const int col = sz_col(cc / SZ_COLS, cc % SZ_COLS);
      if (col < 0 || col >= d.coarse_k) return;
      const int e = e0 + row;
      d.SZc[(int64_t)col * d.nA + e] = s + lam * d.DA[e] * d.Zc[(int64_t)col * d.nA + e];
    });
  } else {
    const int v = blockIdx.x - d.ng, e0 = a_grp(d, 2, v);
    T zg[3][CPL], zc[CD][CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      zg[0][q] = zr[(int64_t)e0 * SZ_COLS + q];
      zg[1][q] = zr[(int64_t)(e0 + 1) * SZ_COLS + q];
      zg[2][q] = 0;
#pragma unroll
      for (int k = 0; k < CD; ++k) zc[k][q] = 0;
    }
    double acc[2][CPL];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int q = 0; q < CPL; ++q) acc[k][q] = 0;
    for (int j = d.vpm_off[v] + rs; j < d.vpm_off[v + 1]; j += R) {
      const int i = d.vpm[j];
      sz_rec_cols<5, 1, T, CD>((const T*)d.frec[5] + (int64_t)i * Slot<5, CD>::STRIDE, zc, zg, sl + (int64_t)d.ffeat[5][i] * 4 * SZ_COLS, acc);
    }
    sz_block_sum<2, L, CPL>(acc, lds, [&](int row, int cc, double s) {
      const int col = sz_col(cc / SZ_COLS, cc % SZ_COLS);
      if (col < 0 || col >= d.coarse_k) return;
      const int e = e0 + row;
      d.SZc[(int64_t)col * d.nA + e] = s + lam * d.DA[e] * d.Zc[(int64_t)col * d.nA + e];
    });
  }
}

// ---------------------------------------------------------------------------
// Deterministic product, second pass: y = J_a^T (J_a x - J_f s_f) row by row, with s_f
// from the first pass.  One workgroup per camera, plane or VP walks that block's records
// (the camera-major copies and the group member lists, as the S Z sweeps do), one record
// per lane with FP64 sums, and reduces them with a fixed butterfly and a fixed sum over
// its wavefronts: the order of every addition is set by the problem, not by scheduling.
// lambda D x is added by k_pcg_q.
template <typename T, int CD> __global__ __launch_bounds__(256) void k_det_cam(Dev d, const double* done) {
  __shared__ double lds[4 * CD];
  if (done && *done != 0.0) return;
  constexpr int R = 256;
  const int c = d.cam_order[blockIdx.x], rs = threadIdx.x;
  const T* x = (const T*)d.xT;
  const T* sp = (const T*)d.sdp;
  const T* sl = (const T*)d.sdl;
  T zc[CD][1], z0[3][1];
#pragma unroll
  for (int k = 0; k < CD; ++k) zc[k][0] = x[CD * c + k];
#pragma unroll
  for (int k = 0; k < 3; ++k) z0[k][0] = 0;
  double acc[CD][1];
#pragma unroll
  for (int k = 0; k < CD; ++k) acc[k][0] = 0;
  auto plane_x = [&](int fam, int g, T (&zg)[3][1]) {
    const int o = a_grp(d, fam == 3 ? Fam<3, CD>::GT : Fam<4, CD>::GT, g);
#pragma unroll
    for (int k = 0; k < 3; ++k) zg[k][0] = x[o + k];
  };
  if (d.fn[1])
    for (int j = d.po_off[c] + rs; j < d.po_off[c + 1]; j += R) {
      const int f = d.cmfeat[1][j];
      sz_rec_cols<1, 0, T, CD>((const T*)d.cmrec[1] + (int64_t)j * Slot<1, CD>::STRIDE, zc, z0, sp + 3 * (int64_t)f, acc, 1);
      const int k = d.cmal[1][j];
      if (k >= 0) {
        T zg[3][1];
        plane_x(3, d.cmgrp[3][k], zg);
        sz_rec_cols<3, 0, T, CD>((const T*)d.cmrec[3] + (int64_t)k * Slot<3, CD>::STRIDE, zc, zg, sp + 3 * (int64_t)f, acc, 1);
      }
    }
  if (d.fn[6])
    for (int j = d.px_off[c] + rs; j < d.px_off[c + 1]; j += R)
      for (int64_t i = d.px_start[j]; i < d.px_start[j] + d.px_cnt[j]; ++i)
        sz_rec_cols<6, 0, T, CD>((const T*)d.frec[6] + i * Slot<6, CD>::STRIDE, zc, z0, sp + 3 * (int64_t)d.ffeat[6][i], acc, 1);
  if (d.fn[2])
    for (int j = d.lo_off[c] + rs; j < d.lo_off[c + 1]; j += R) {
      const int f = d.cmfeat[2][j];
      sz_rec_cols<2, 0, T, CD>((const T*)d.cmrec[2] + (int64_t)j * Slot<2, CD>::STRIDE, zc, z0, sl + 4 * (int64_t)f, acc, 1);
      const int k = d.cmal[2][j];
      if (k >= 0) {
        T zg[3][1];
        plane_x(4, d.cmgrp[4][k], zg);
        sz_rec_cols<4, 0, T, CD>((const T*)d.cmrec[4] + (int64_t)k * Slot<4, CD>::STRIDE, zc, zg, sl + 4 * (int64_t)f, acc, 1);
      }
    }
  if (d.fn[7])
    for (int j = d.lx_off[c] + rs; j < d.lx_off[c + 1]; j += R)
      for (int64_t i = d.lx_start[j]; i < d.lx_start[j] + d.lx_cnt[j]; ++i)
        sz_rec_cols<7, 0, T, CD>((const T*)d.frec[7] + i * Slot<7, CD>::STRIDE, zc, z0, sl + 4 * (int64_t)d.ffeat[7][i], acc, 1);
  double* y = d.mv_part;
  sz_block_sum<CD, 1, 1>(acc, lds, [&](int row, int, double v) { y[CD * c + row] = v; });
}

template <typename T, int CD> __global__ __launch_bounds__(256) void k_det_grp(Dev d, const double* done) {
  __shared__ double lds[4 * 3];
  if (done && *done != 0.0) return;
  constexpr int R = 256;
  const int rs = threadIdx.x;
  const T* x = (const T*)d.xT;
  const T* sp = (const T*)d.sdp;
  const T* sl = (const T*)d.sdl;
  double* y = d.mv_part;
  if ((int)blockIdx.x < d.ng) {
    const int g = blockIdx.x, e0 = a_grp(d, 1, g);
    T zg[3][1];
#pragma unroll
    for (int k = 0; k < 3; ++k) zg[k][0] = x[e0 + k];
    double acc[3][1] = {{0}, {0}, {0}};
    if (d.fn[3] || d.fn[8])
      for (int j = d.plp_off[g] + rs; j < d.plp_off[g + 1]; j += R) {
        const int f = d.plp[j];
        for (int64_t i = d.foff[3][f]; i < d.foff[3][f + 1]; ++i) {
          if (d.fgrp[3][i] != g) continue;
          T zc[CD][1];
#pragma unroll
          for (int k = 0; k < CD; ++k) zc[k][0] = x[CD * d.fcam[3][i] + k];
          sz_rec_cols<3, 1, T, CD>((const T*)d.frec[3] + i * Slot<3, CD>::STRIDE, zc, zg, sp + 3 * (int64_t)f, acc, 1);
        }
        for (int64_t i = d.foff[8][f]; i < d.foff[8][f + 1]; ++i) {
          if (d.fgrp[8][i] != g) continue;
          T zc[CD][1];
#pragma unroll
          for (int k = 0; k < CD; ++k) zc[k][0] = 0;
          sz_rec_cols<8, 1, T, CD>((const T*)d.frec[8] + i * Slot<8, CD>::STRIDE, zc, zg, sp + 3 * (int64_t)f, acc, 1);
        }
      }
    if (d.fn[4])
      for (int j = d.pll_off[g] + rs; j < d.pll_off[g + 1]; j += R) {
        const int f = d.pll[j];
        for (int64_t i = d.foff[4][f]; i < d.foff[4][f + 1]; ++i) {
          T zc[CD][1];
#pragma unroll
          for (int k = 0; k < CD; ++k) zc[k][0] = x[CD * d.fcam[4][i] + k];
          sz_rec_cols<4, 1, T, CD>((const T*)d.frec[4] + i * Slot<4, CD>::STRIDE, zc, zg, sl + 4 * (int64_t)f, acc, 1);
        }
      }
    sz_block_sum<3, 1, 1>(acc, lds, [&](int row, int, double v) { y[e0 + row] = v; });
  } else {
    const int v = blockIdx.x - d.ng, e0 = a_grp(d, 2, v);
    T zg[3][1], zc[CD][1];
    zg[0][0] = x[e0];
    zg[1][0] = x[e0 + 1];
    zg[2][0] = 0;
#pragma unroll
    for (int k = 0; k < CD; ++k) zc[k][0] = 0;
    double acc[2][1] = {{0}, {0}};
    for (int j = d.vpm_off[v] + rs; j < d.vpm_off[v + 1]; j += R) {
      const int i = d.vpm[j];
      sz_rec_cols<5, 1, T, CD>((const T*)d.frec[5] + (int64_t)i * Slot<5, CD>::STRIDE, zc, zg, sl + 4 * (int64_t)d.ffeat[5][i], acc, 1);
    }
    sz_block_sum<2, 1, 1>(acc, lds, [&](int row, int, double w) { y[e0 + row] = w; });
  }
}

template <typename T, int CD> void launch_det_rows(const Dev& d, const double* done, hipStream_t s) {
  if (d.nc) k_det_cam<T, CD><<<d.nc, 256, 0, s>>>(d, done);
  if (d.ng + d.nv) k_det_grp<T, CD><<<d.ng + d.nv, 256, 0, s>>>(d, done);
}

template <typename T, int CD, int L, int CPL>
__global__ __launch_bounds__(256) void k_sz_shape(Dev d, const T* Zr, const T* sfp, const T* sfl, double lam);
__global__ void k_sz_shape_fin(Dev d, double lam);

template <typename T, int CD, int L, int CPL> static void launch_sz_out(const Dev& d, const T* Zr, const T* sfp, const T* sfl, double lambda, hipStream_t s) {
  if (d.nc) k_sz_cam<T, CD, L, CPL><<<d.nc, 256, 0, s>>>(d, Zr, sfp, sfl, lambda);
  if (d.ng + d.nv) k_sz_grp<T, CD, L, CPL><<<d.ng + d.nv, 256, 0, s>>>(d, Zr, sfp, sfl, lambda);
  if (d.ns) {
    launch_zero(d.shsz, (size_t)d.ns * SH_DOF * SZ_COLS * SZ_PANELS * sizeof(double), s);
    if (d.n_shch) k_sz_shape<T, CD, L, CPL><<<d.n_shch, 256, 0, s>>>(d, Zr, sfp, sfl, lambda);
    k_sz_shape_fin<<<d.ns, 128, 0, s>>>(d, lambda);
  }
}

template <typename T, int CD> static void launch_sz(const Dev& d, double lambda, hipStream_t s) {
  T* Zr = (T*)d.szr;
  T* sfp = (T*)d.szfp;
  T* sfl = (T*)d.szfl;
  const SzPanels P = sz_panels(d);
  // no VP 3-vector records: the gauge panel's s_f in closed form, no record sweep for it
  // the closed form needs J z = 0 for the gauge directions: not so for the VP
  // 3-vector (turns with the world) nor for the metric 3D point-to-plane distance
  // (scales with the world)
  const bool closed = d.fn[5] == 0 && d.fn[8] == 0 && d.ns == 0;
  k_sz_rows<T><<<nblk(P.z * SZ_PANELS, 256), 256, 0, s>>>(d, Zr, closed ? 1 : 0);
  for (int pn = 0; pn < SZ_PANELS && sz_col(pn, 0) < d.coarse_k; ++pn) {
    T *zp = Zr + pn * P.z, *pp = sfp + pn * P.p, *lp = sfl + pn * P.l;
    if (pn == 0 && closed) {
      if (d.np + d.nl) k_sz_gauge_feat<T><<<nblk(d.np + d.nl, 256), 256, 0, s>>>(d, pp, lp, lambda);
      continue;
    }
    if (d.n_tiles) k_sz_feat_wave<T, CD><<<(int)std::min<int64_t>(4 * (int64_t)d.n_mv_wg, nblk(d.n_tiles, 4)), 256, 0, s>>>(d, zp, pp, lp);
    // one wavefront per large feature
    if (d.n_bigp) k_sz_feat_big<T, CD, 3><<<std::min(nblk(d.n_bigp, 4), 4096u), 256, 0, s>>>(d, zp, pp, d.bigp, d.n_bigp);
    if (d.n_bigl) k_sz_feat_big<T, CD, 4><<<std::min(nblk(d.n_bigl, 4), 4096u), 256, 0, s>>>(d, zp, lp, d.bigl, d.n_bigl);
  }
  static_assert(SZ_PANELS == 2, "one or two panels");
  if (d.coarse_k <= COARSE_GAUGE) launch_sz_out<T, CD, SZ_LANES, SZ_COLS / SZ_LANES>(d, Zr, sfp, sfl, lambda, s);
  else launch_sz_out<T, CD, 2 * SZ_LANES, SZ_COLS / SZ_LANES>(d, Zr, sfp, sfl, lambda, s);
}

void launch_coarse_setup(const Dev& d, double lambda, hipStream_t s) {
  BA_DISPATCH_T_CD(d, launch_sz<T, CD>(d, lambda, s));
  // inter-group relations touch no feature: their part of S Z is U_rel Z in the group
  // rows, for the gauge columns too (the closed form covers the feature records only)
  launch_rel_sz(d, s);
  double* E = d.Ztb + COARSE_K;  // K x K scratch after Z^T b
  k_coarse_e<<<COARSE_K * COARSE_K, 256, 0, s>>>(d, E);
  k_coarse_inv<<<1, 512, 0, s>>>(d, E);
}


// ---------------------------------------------------------------------------
// back-substitution h_f = -(V_f + lambda D_f)^-1 (g_f + J_f^T J_a h_a), and the
// model-decrease terms h.g and sum |J h|^2 (FP64 accumulation)
// |J x_a + J_f h|^2 of one record (FP64 sums): the slot loaded whole, or a row at a time
// for the surface-group families
template <int FAM, typename T, int CD, int NF>
__device__ __forceinline__ double rec_jh2(const Dev& d, int64_t i, const T* x, const T (&h)[NF]) {
  using SL = Slot<FAM, CD>;
  using F = Fam<FAM, CD>;
  const T* sl = (const T*)d.frec[FAM] + i * SL::STRIDE;
  double jh2 = 0;
  if constexpr (F::GT == 3) {
    const T* xc = x + CD * d.fcam[FAM][i];
    const T* xg = x + a_grp(d, 3, d.fgrp[FAM][i]);
#pragma unroll 1
    for (int row = 0; row < SL::ROWS; ++row) {
      double t = 0;
#pragma unroll
      for (int k = 0; k < SL::NC; ++k) t += (double)sl[SL::OC + row * SL::NC + k] * (double)xc[k];
#pragma unroll
      for (int k = 0; k < SL::NG; ++k) t += (double)sl[SL::OG + row * SL::NG + k] * (double)xg[k];
#pragma unroll
      for (int a = 0; a < NF; ++a) t += (double)sl[SL::OF + row * NF + a] * (double)h[a];
      jh2 += t * t;
    }
  } else {
    T v[SL::STRIDE];
    load_vec(sl, v);
    T xc[SL::NC > 0 ? SL::NC : 1], xg[SL::NG > 0 ? SL::NG : 1];
    if constexpr (SL::NC > 0) {
      const T* xp = x + CD * d.fcam[FAM][i];
#pragma unroll
      for (int k = 0; k < SL::NC; ++k) xc[k] = xp[k];
    }
    if constexpr (SL::NG > 0) {
      const T* xp = x + a_grp(d, F::GT, d.fgrp[FAM][i]);
#pragma unroll
      for (int k = 0; k < SL::NG; ++k) xg[k] = xp[k];
    }
#pragma unroll
    for (int row = 0; row < SL::ROWS; ++row) {
      double t = 0;
#pragma unroll
      for (int k = 0; k < SL::NC; ++k) t += (double)v[SL::OC + row * SL::NC + k] * (double)xc[k];
#pragma unroll
      for (int k = 0; k < SL::NG; ++k) t += (double)v[SL::OG + row * SL::NG + k] * (double)xg[k];
#pragma unroll
      for (int a = 0; a < NF; ++a) t += (double)v[SL::OF + row * NF + a] * (double)h[a];
      jh2 += t * t;
    }
  }
  return jh2;
}

template <int FAM, typename T, int CD, int NF>
__device__ __forceinline__ double wave_jh2(const Dev& d, int64_t b, int n, const T* x, const T (&h)[NF], int& j0, int lane) {
  double jh2 = 0;
  for (int r = (lane - j0 % 64 + 64) % 64; r < n; r += 64) jh2 += rec_jh2<FAM, T, CD, NF>(d, b + r, x, h);
  j0 += n;
  return jh2;
}

// back-substitution of one feature larger than a tile (or a line on a shape), one
// wavefront: q = J_f^T J_a h_a summed across it, h_f = -(V_f + lambda D_f)^-1 (g_f + q)
// stored and g_f . h_f added by lane 0, |J h|^2 of each lane's records added on that lane
template <typename T, int CD, int NF>
__device__ __forceinline__ void backsub_feature_wave(const Dev& d, int f, const T* x, int lane, double& gh, double& jh2) {
  constexpr int F0 = NF == 3 ? 1 : 2, F1 = NF == 3 ? 3 : 4, F2 = NF == 3 ? 6 : 5, F3 = NF == 3 ? 8 : 7;
  constexpr int FS = NF == 3 ? 9 : 10;
  int64_t b[5];
  int n[5];
  auto range = [&](int k, int F) {
    if (d.fn[F]) {
      b[k] = d.foff[F][f];
      n[k] = (int)(d.foff[F][f + 1] - b[k]);
    } else {
      b[k] = 0;
      n[k] = 0;
    }
  };
  range(0, F0); range(1, F1); range(2, F2); range(3, F3); range(4, FS);
  T q[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) q[k] = 0;
  int j0 = 0;
  wave_first<F0, T, CD, NF>(d, b[0], n[0], x, j0, lane, q);
  wave_first<F1, T, CD, NF>(d, b[1], n[1], x, j0, lane, q);
  wave_first<F2, T, CD, NF>(d, b[2], n[2], x, j0, lane, q);
  wave_first<F3, T, CD, NF>(d, b[3], n[3], x, j0, lane, q);
  wave_first<FS, T, CD, NF>(d, b[4], n[4], x, j0, lane, q);
  const T* g = (const T*)(NF == 3 ? d.gp : d.gl) + (int64_t)NF * f;
#pragma unroll
  for (int k = 0; k < NF; ++k) q[k] = -(wave_sum(q[k]) + g[k]);
  T h[NF];
  apply_vinv<T, NF>(d, f, q, h);
  if (lane == 0) {
    double* ho = (NF == 3 ? d.hp : d.hl) + (int64_t)NF * f;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      ho[k] = (double)h[k];
      gh += (double)g[k] * (double)h[k];
    }
  }
  j0 = 0;
  jh2 += wave_jh2<F0, T, CD, NF>(d, b[0], n[0], x, h, j0, lane);
  jh2 += wave_jh2<F1, T, CD, NF>(d, b[1], n[1], x, h, j0, lane);
  jh2 += wave_jh2<F2, T, CD, NF>(d, b[2], n[2], x, h, j0, lane);
  jh2 += wave_jh2<F3, T, CD, NF>(d, b[3], n[3], x, h, j0, lane);
  jh2 += wave_jh2<FS, T, CD, NF>(d, b[4], n[4], x, h, j0, lane);
}


// |J h|^2 of one record given t = J_a h_a and the broadcast h_f (FP64 sum)
template <int FAM, typename T, int CD>
__device__ __forceinline__ double bs_record(const T (&v)[MaxSlot<CD>::V], const T (&t)[4], const T (&h)[4]) {
  using SL = Slot<FAM, CD>;
  double acc = 0;
#pragma unroll
  for (int row = 0; row < SL::ROWS; ++row) {
    double u = (double)t[row];
#pragma unroll
    for (int a = 0; a < SL::NF; ++a) u += (double)v[SL::OF + row * SL::NF + a] * (double)h[a];
    acc += u * u;
  }
  return acc;
}

template <int FAM, typename T, int CD>
__device__ __forceinline__ double bs_record_reload(const Dev& d, int64_t i, const T (&t)[4], const T (&h)[4]) {
  using SL = Slot<FAM, CD>;
  T v[MaxSlot<CD>::V];
  const double2* q2 = reinterpret_cast<const double2*>((const T*)d.frec[FAM] + i * SL::STRIDE);
#pragma unroll
  for (int k = 0; k < SL::STRIDE / 2; ++k) {
    double2 a = q2[k];
    v[2 * k] = a.x; v[2 * k + 1] = a.y;
  }
  return bs_record<FAM, T, CD>(v, t, h);
}

// Back-substitution over the product's wavefront tiles: t = J_a h_a and
// q_f = sum J_f^T t as in the product, h_f = -(V_f + lambda D_f)^-1 (g_f + q_f) on the
// feature's last lane, then |J_a h_a + J_f h_f|^2 per record; per-workgroup sums of
// g_f . h_f and |J h|^2 go to d.red
// FP32: at most 128 VGPRs (4 wavefronts per SIMD; 132 without the bound, 3 per SIMD);
// FP64 would spill under it
template <typename T> constexpr int backsub_min_waves() { return sizeof(T) == 4 ? 4 : 1; }

template <typename T, int CD> __global__ __launch_bounds__(256, backsub_min_waves<T>()) void k_backsub_wave(Dev d) {
  __shared__ double lds[2 * 5];
  // each lane's (g.h, |J h|^2) sums in LDS rather than in registers held across the tiles
  __shared__ double bs_acc[2 * 256];
  const T* x = (const T*)d.xT;
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  double* acc = bs_acc + 2 * threadIdx.x;
  acc[0] = 0;
  acc[1] = 0;
  for (int tile = blockIdx.x * nw + (threadIdx.x >> 6); tile < d.n_tiles; tile += gridDim.x * nw) {
    const int4 tl = d.tiles[tile];
    const int fb = tl.z;
    const bool active = lane < tl.y;
    const bool ptile = tile < d.n_ptiles;
    int4 w4 = make_int4(0, 0, 0, -1);
    if (active) w4 = d.wrec[tl.x + lane];
    const int fam = (int)((uint32_t)w4.x >> 28), lf = w4.w;
    const int64_t i = (int64_t)((uint32_t)w4.x & 0x0fffffffu);
    const int next = __shfl_down(lf, 1, 64);
    const bool last = lf >= 0 && (lane == 63 || next != lf);
    T Mi[10], g[4] = {0, 0, 0, 0};
    bool mflag = false;
    if (last) {
      const int f = fb + lf;
      mflag = (ptile ? d.flp[f] : d.fll[f]) != 0;
      if (ptile) {
        const T* M = (const T*)d.Vip + 6 * (int64_t)f;
#pragma unroll
        for (int k = 0; k < 6; ++k) Mi[k] = M[k];
        const T* gp = (const T*)d.gp + 3 * (int64_t)f;
#pragma unroll
        for (int k = 0; k < 3; ++k) g[k] = gp[k];
      } else {
        const T* M = (const T*)d.Vil + 10 * (int64_t)f;
#pragma unroll
        for (int k = 0; k < 10; ++k) Mi[k] = M[k];
        const T* gl = (const T*)d.gl + 4 * (int64_t)f;
#pragma unroll
        for (int k = 0; k < 4; ++k) g[k] = gl[k];
      }
    }
    T v[MaxSlot<CD>::V];
    T t[4] = {0, 0, 0, 0};
    T q[4] = {0, 0, 0, 0};
    int ac = 0, ag = 0;
    if (active) {
      switch (fam) {
        case 1: tile_phase_a<1, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 2: tile_phase_a<2, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 3: tile_phase_a<3, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 4: tile_phase_a<4, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 5: tile_phase_a<5, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 6: tile_phase_a<6, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 7: tile_phase_a<7, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 8: tile_phase_a<8, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
        case 9: tile_phase_a<9, T, CD>(d, i, w4.y, w4.z, x, q, v, t, ac, ag); break;
      }
    }
    const int prev = __shfl_up(lf, 1, 64);
    const unsigned long long heads = __ballot(lf >= 0 && (lane == 0 || prev != lf));
    const int start = lf >= 0 ? 63 - __builtin_clzll(heads & ((2ull << lane) - 1ull)) : lane;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const bool take = lane - off >= start;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (a == 3 && ptile) continue;
        const T o = __shfl_up(q[a], off, 64);
        if (take) q[a] += o;
      }
    }
    const unsigned long long lasts = __ballot(last);
    T h[4] = {0, 0, 0, 0};
    if (last) {
      T rhs[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) rhs[a] = -(q[a] + g[a]);
      const int f = fb + lf;
      if (ptile) feature_solve<T, 3>(d, f, mflag, Mi, rhs, h);
      else feature_solve<T, 4>(d, f, mflag, Mi, rhs, h);
      const int nfa = ptile ? 3 : 4;
      double* ho = (ptile ? d.hp : d.hl) + (int64_t)nfa * f;
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (a < nfa) {
          ho[a] = (double)h[a];
          acc[0] += (double)g[a] * (double)h[a];
        }
    }
    const int src = lf >= 0 ? __builtin_ctzll(lasts & (~0ull << lane)) : lane;
#pragma unroll
    for (int a = 0; a < 4; ++a) h[a] = __shfl(h[a], src, 64);
    if (active) {
      if constexpr (sizeof(T) == 4) {
        switch (fam) {
          case 1: acc[1] += bs_record<1, T, CD>(v, t, h); break;
          case 2: acc[1] += bs_record<2, T, CD>(v, t, h); break;
          case 3: acc[1] += bs_record<3, T, CD>(v, t, h); break;
          case 4: acc[1] += bs_record<4, T, CD>(v, t, h); break;
          case 5: acc[1] += bs_record<5, T, CD>(v, t, h); break;
          case 6: acc[1] += bs_record<6, T, CD>(v, t, h); break;
          case 7: acc[1] += bs_record<7, T, CD>(v, t, h); break;
          case 8: acc[1] += bs_record<8, T, CD>(v, t, h); break;
          case 9: acc[1] += bs_record<9, T, CD>(v, t, h); break;
        }
      } else {
        switch (fam) {
          case 1: acc[1] += bs_record_reload<1, T, CD>(d, i, t, h); break;
          case 2: acc[1] += bs_record_reload<2, T, CD>(d, i, t, h); break;
          case 3: acc[1] += bs_record_reload<3, T, CD>(d, i, t, h); break;
          case 4: acc[1] += bs_record_reload<4, T, CD>(d, i, t, h); break;
          case 5: acc[1] += bs_record_reload<5, T, CD>(d, i, t, h); break;
          case 6: acc[1] += bs_record_reload<6, T, CD>(d, i, t, h); break;
          case 7: acc[1] += bs_record_reload<7, T, CD>(d, i, t, h); break;
          case 8: acc[1] += bs_record_reload<8, T, CD>(d, i, t, h); break;
          case 9: acc[1] += bs_record_reload<9, T, CD>(d, i, t, h); break;
        }
      }
    }
  }
  // features whose records do not fit one tile (and features on a shape) are
  // k_backsub_big's
  double vals[2] = {acc[0], acc[1]};
  double* o = block_sum_arr<double, 2>(vals, lds);
  if (threadIdx.x == 0) { d.red[2 * blockIdx.x] = o[0]; d.red[2 * blockIdx.x + 1] = o[1]; }
}

// back-substitution of the large features, one wavefront each; its workgroups' (g.h,
// |J h|^2) partials follow k_backsub_wave's in d.red from slot red0
template <typename T, int CD> __global__ __launch_bounds__(256) void k_backsub_big(Dev d, int red0) {
  __shared__ double lds[2 * 5];
  const T* x = (const T*)d.xT;
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  double gh = 0, jh2 = 0;
  for (int k = blockIdx.x * nw + (threadIdx.x >> 6); k < d.n_bigp + d.n_bigl; k += gridDim.x * nw) {
    if (k < d.n_bigp) backsub_feature_wave<T, CD, 3>(d, d.bigp[k], x, lane, gh, jh2);
    else backsub_feature_wave<T, CD, 4>(d, d.bigl[k - d.n_bigp], x, lane, gh, jh2);
  }
  double vals[2] = {gh, jh2};
  double* o = block_sum_arr<double, 2>(vals, lds);
  if (threadIdx.x == 0) {
    d.red[2 * (red0 + blockIdx.x)] = o[0];
    d.red[2 * (red0 + blockIdx.x) + 1] = o[1];
  }
}

// J h over the records of the features is covered by the feature pass (the
// inter-group relations, which have no feature, are added by launch_rel_md); this
// adds g_a . h_a and sums the partials
__global__ __launch_bounds__(1024) void k_md_final(Dev d, int nparts) {
  __shared__ double lds[2 * 17];
  double v[2] = {0, 0};
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) { v[0] += d.red[2 * i]; v[1] += d.red[2 * i + 1]; }
  for (int k = threadIdx.x; k < d.nA; k += blockDim.x) v[0] += d.gA[k] * d.x[k];
  double* o = block_sum_arr<double, 2>(v, lds);
  if (threadIdx.x == 0) { d.scal[SC_GH] = o[0]; d.scal[SC_JH2] = o[1]; }
}

void launch_backsub(const Dev& d, hipStream_t s) {
  // the large features' workgroups take at most half of the partial slots
  const int nbig = d.n_bigp + d.n_bigl;
  const int gbig = nbig ? (int)std::min<int64_t>(std::min<int64_t>(nblk(nbig, 4), 64), d.n_red_max / 2) : 0;
  const int nwg = (int)std::max<int64_t>(1, std::min<int64_t>(4 * (int64_t)d.n_mv_wg, d.n_red_max - gbig));
  BA_DISPATCH_T_CD(d, {
    k_to_T<T><<<nblk(d.nA, 256), 256, 0, s>>>(d.x, d.xT, d.nA);
    k_backsub_wave<T, CD><<<nwg, 256, 0, s>>>(d);
    if (gbig) k_backsub_big<T, CD><<<gbig, 256, 0, s>>>(d, nwg);
  });
  k_md_final<<<1, 1024, 0, s>>>(d, nwg + gbig);
  launch_rel_md(d, s);
}

// ---------------------------------------------------------------------------
// retraction in FP64: candidate = current [+] (h_a, h_f)
__device__ void so3_exp(const double* w, double* E) {
  const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double th = sqrt(th2);
  double a, b;
  if (th < 1e-8) { a = 1.0 - th2 / 6.0; b = 0.5 - th2 / 24.0; }
  else { a = sin(th) / th; b = (1.0 - cos(th)) / th2; }
  const double W[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
  double W2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) W2[3 * i + j] = W[3 * i] * W[j] + W[3 * i + 1] * W[3 + j] + W[3 * i + 2] * W[6 + j];
  for (int k = 0; k < 9; ++k) E[k] = (k % 4 == 0 ? 1.0 : 0.0) + a * W[k] + b * W2[k];
}

// tangent basis of the sphere at n: b1 = normalise(e_k - (e_k.n) n), k = argmin |n_k|, b2 = n x b1
__device__ void s2_basis(const double* n, double* b1, double* b2) {
  int k = 0;
  if (fabs(n[1]) < fabs(n[k])) k = 1;
  if (fabs(n[2]) < fabs(n[k])) k = 2;
  double e[3] = {0, 0, 0};
  e[k] = 1.0;
  const double en = n[k];
  for (int i = 0; i < 3; ++i) b1[i] = e[i] - en * n[i];
  const double nb = sqrt(b1[0] * b1[0] + b1[1] * b1[1] + b1[2] * b1[2]);
  for (int i = 0; i < 3; ++i) b1[i] /= nb;
  cross3(n, b1, b2);
}

__device__ void s2_retract(const double* n, const double* b1, const double* b2, double d0, double d1, double* out) {
  if (d0 == 0.0 && d1 == 0.0) {  // no step (a fixed group): unchanged, not renormalised
    for (int i = 0; i < 3; ++i) out[i] = n[i];
    return;
  }
  double v[3];
  for (int i = 0; i < 3; ++i) v[i] = b1[i] * d0 + b2[i] * d1;
  const double th = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  for (int i = 0; i < 3; ++i) out[i] = th < 1e-12 ? n[i] + v[i] : cos(th) * n[i] + sin(th) * v[i] / th;
  const double nn = sqrt(out[0] * out[0] + out[1] * out[1] + out[2] * out[2]);
  for (int i = 0; i < 3; ++i) out[i] /= nn;
}

__global__ void k_retract(Dev d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int CD = d.CD;
  if (i < d.nc) {
    const double* c = d.cam64 + (int64_t)CAM_STRIDE * i;
    double* o = d.cam64n + (int64_t)CAM_STRIDE * i;
    const double* h = d.x + CD * i;
    double E[9];
    so3_exp(h, E);
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) o[3 * r + k] = E[3 * r] * c[k] + E[3 * r + 1] * c[3 + k] + E[3 * r + 2] * c[6 + k];
    for (int r = 0; r < 3; ++r) o[9 + r] = E[3 * r] * c[9] + E[3 * r + 1] * c[10] + E[3 * r + 2] * c[11] + h[3 + r];
    o[12] = c[12] + (CD == 9 ? h[6] : 0.0);
    o[13] = c[13] + (CD == 9 ? h[7] : 0.0);
    o[14] = c[14] + (CD == 9 ? h[8] : 0.0);
    o[15] = 0;
    return;
  }
  int j = i - d.nc;
  if (j < d.np) {
    for (int k = 0; k < 3; ++k) d.pt64n[PT_STRIDE * (int64_t)j + k] = d.pt64[PT_STRIDE * (int64_t)j + k] + d.hp[3 * (int64_t)j + k];
    d.pt64n[PT_STRIDE * (int64_t)j + 3] = 0;
    return;
  }
  j -= d.np;
  if (j < d.nl) {
    const double* L = d.ln64 + (int64_t)LN_STRIDE * j;
    double* o = d.ln64n + (int64_t)LN_STRIDE * j;
    const double* h = d.hl + 4 * (int64_t)j;
    double E[9];
    so3_exp(h, E);
    // U' = U E with U = [u1 u2 u3] (columns stored consecutively)
    for (int col = 0; col < 3; ++col)
      for (int r = 0; r < 3; ++r) o[3 * col + r] = L[r] * E[col] + L[3 + r] * E[3 + col] + L[6 + r] * E[6 + col];
    const double cph = cos(h[3]), sph = sin(h[3]);
    o[9] = L[9] * cph - L[10] * sph;
    o[10] = L[9] * sph + L[10] * cph;
    o[11] = 0;
    return;
  }
  j -= d.nl;
  if (j < d.ng) {
    const double* P = d.pl64 + (int64_t)PL_STRIDE * j;
    double* o = d.pl64n + (int64_t)PL_STRIDE * j;
    const double* h = d.x + d.offPl + 3 * j;
    s2_retract(P, P + 4, P + 7, h[0], h[1], o);
    o[3] = P[3] + h[2];
    s2_basis(o, o + 4, o + 7);
    o[10] = o[11] = 0;
    return;
  }
  j -= d.ng;
  if (j < d.nv) {
    const double* V = d.vp64 + (int64_t)VP_STRIDE * j;
    double* o = d.vp64n + (int64_t)VP_STRIDE * j;
    const double* h = d.x + d.offVp + 2 * j;
    s2_retract(V, V + 4, V + 7, h[0], h[1], o);
    o[3] = 0;
    s2_basis(o, o + 4, o + 7);
    o[10] = o[11] = 0;
  }
}

__global__ void k_shape_retract(Dev d);

void launch_retract(const Dev& d, hipStream_t s) {
  const int n = d.nc + d.np + d.nl + d.ng + d.nv;
  if (n) k_retract<<<nblk(n, 256), 256, 0, s>>>(d);
  if (d.ns) k_shape_retract<<<nblk(d.ns, 64), 64, 0, s>>>(d);
}

__global__ void k_zero(unsigned char* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}
// ---------------------------------------------------------------------------
// feature statistics for the reliability-aware refinement

// smallest eigenvalue of a symmetric N x N matrix (overwritten) by cyclic Jacobi
// rotations in FP64, until the off-diagonal mass is below 1e-30 of the diagonal's
template <int N> __device__ double sym_min_eig(double (&A)[N][N]) {
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, dia = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      dia += A[i][i] * A[i][i];
#pragma unroll
      for (int j = i + 1; j < N; ++j) off += A[i][j] * A[i][j];
    }
    if (!(off > 1e-30 * dia)) break;
#pragma unroll
    for (int p = 0; p < N; ++p)
#pragma unroll
      for (int q = p + 1; q < N; ++q) {
        const double apq = A[p][q];
        if (fabs(apq) < 1e-300) continue;
        // rotation angle that zeroes A[p][q]: t = tan(phi), the smaller root
        const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = fabs(th) > 1e150 ? 0.5 / th : (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
      }
  }
  double m = A[0][0];
#pragma unroll
  for (int i = 1; i < N; ++i) m = fmin(m, A[i][i]);
  return m;
}

// one thread per point (NF 3) or line (NF 4): its observation records (R1 / R2)
// in the quadratic part of their loss, their count, and sigma from the feature block
template <typename T, int NF> __global__ __launch_bounds__(256) void k_feat_stats(Dev d, int32_t* nact, int32_t* nobs,
                                                                                  double* sig) {
  constexpr int FAM = NF == 3 ? 1 : 2;
  constexpr int NS = NF * (NF + 1) / 2;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= (NF == 3 ? d.np : d.nl)) return;
  const int32_t r0 = d.foff[FAM][f], r1 = d.foff[FAM][f + 1];
  const double s2 = d.lscale[FAM] * d.lscale[FAM];
  int act = 0;
  double dsum = 0.0;
  for (int32_t r = r0; r < r1; ++r) {
    double res[4];
    residual64<FAM>(d, r, d.cam64, d.pt64, d.ln64, d.pl64, d.vp64, d.sh64, res);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < Fam<FAM, 9>::ROWS; ++k) s += res[k] * res[k];
    if (d.lkind[FAM] == 0 || s <= s2) ++act;
    if constexpr (NF == 3) {
      const double* c = d.cam64 + (int64_t)CAM_STRIDE * d.fcam[FAM][r];
      const double* X = d.pt64 + (int64_t)PT_STRIDE * f;
      double e = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double ck = -(c[k] * c[9] + c[3 + k] * c[10] + c[6 + k] * c[11]);
        e += (X[k] - ck) * (X[k] - ck);
      }
      dsum += sqrt(e);
    }
  }
  const T* P = (const T*)(NF == 3 ? d.Vp : d.Vl) + (int64_t)NS * f;
  double A[NF][NF];
#pragma unroll
  for (int i = 0; i < NF; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) A[i][j] = (double)P[sym<NF>(i, j)];
  const double lam = sym_min_eig<NF>(A);
  double sigma = lam > 0.0 ? 1.0 / sqrt(lam) : INFINITY;
  if constexpr (NF == 3) sigma = r1 > r0 ? sigma / (dsum / (double)(r1 - r0)) : INFINITY;
  nact[f] = act;
  nobs[f] = r1 - r0;
  sig[f] = sigma;
}

void launch_feature_stats(const Dev& d, int32_t* n_active, int32_t* n_obs, double* sigma, int nf, hipStream_t s) {
  const int n = nf == 3 ? d.np : d.nl;
  if (!n) return;
  if (nf == 3) {
    if (d.fp64) k_feat_stats<double, 3><<<nblk(n, 256), 256, 0, s>>>(d, n_active, n_obs, sigma);
    else k_feat_stats<float, 3><<<nblk(n, 256), 256, 0, s>>>(d, n_active, n_obs, sigma);
  } else {
    if (d.fp64) k_feat_stats<double, 4><<<nblk(n, 256), 256, 0, s>>>(d, n_active, n_obs, sigma);
    else k_feat_stats<float, 4><<<nblk(n, 256), 256, 0, s>>>(d, n_active, n_obs, sigma);
  }
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes) k_zero<<<256, 256, 0, s>>>((unsigned char*)p, bytes);
}

// ---------------------------------------------------------------------------
// surface groups (App. B): their blocks of the reduced system, one workgroup per shape

// U_ss, g_s of one record (shape columns, one row at a time)
template <int FAM, typename T, int CD>
__device__ __forceinline__ void shape_a_rows(const Dev& d, int64_t i, T (&U)[SH_DOF * (SH_DOF + 1) / 2], T (&g)[SH_DOF]) {
  using SL = Slot<FAM, CD>;
  const T* sl = (const T*)d.frec[FAM] + i * SL::STRIDE;
  const T* res = (const T*)d.fres[FAM] + i * SL::ROWS;
#pragma unroll 1
  for (int row = 0; row < SL::ROWS; ++row) {
    T jg[SH_DOF];
#pragma unroll
    for (int k = 0; k < SH_DOF; ++k) jg[k] = sl[SL::OG + row * SH_DOF + k];
    const T rr = res[row];
#pragma unroll
    for (int a = 0; a < SH_DOF; ++a) {
      g[a] += jg[a] * rr;
#pragma unroll
      for (int b = a; b < SH_DOF; ++b) U[sym<SH_DOF>(a, b)] += jg[a] * jg[b];
    }
  }
}

// Each pass runs one workgroup per chunk of at most SH_CHUNK members of a shape (a large
// shape has tens of thousands of points), sums its chunk over the workgroup and adds the
// sums to the shape's FP64 accumulator with one atomic each; a per-shape kernel then
// writes the blocks.  The accumulators are cleared first.
template <typename T, int CD, bool B> __global__ __launch_bounds__(256) void k_shape_chunk(Dev d) {
  constexpr int NS = SH_DOF * (SH_DOF + 1) / 2, K = NS + SH_DOF;
  static_assert(K == SH_ACC, "accumulator layout");
  __shared__ T lds[(4 + 1) * K];
  const int4 ch = d.shch[blockIdx.x];  // (shape, first member, members, kind)
  T acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0;
  T(&U)[NS] = *reinterpret_cast<T(*)[NS]>(acc);
  T(&g)[SH_DOF] = *reinterpret_cast<T(*)[SH_DOF]>(acc + NS);
  for (int j = ch.y + threadIdx.x; j < ch.y + ch.z; j += blockDim.x) {
    if (ch.w == 0) {
      const int f = d.shp[j];
      if constexpr (B) {
        T W[SH_DOF][3];
#pragma unroll
        for (int a = 0; a < SH_DOF; ++a) W[a][0] = W[a][1] = W[a][2] = 0;
        for (int64_t i = d.foff[9][f]; i < d.foff[9][f + 1]; ++i) addW_rows<9, 1, T, CD, SH_DOF, 3>(d, i, W);
        pair_contrib<T, SH_DOF, 3>(d, f, W, acc, acc + NS);
      } else {
        for (int64_t i = d.foff[9][f]; i < d.foff[9][f + 1]; ++i) shape_a_rows<9, T, CD>(d, i, U, g);
      }
    } else {
      const int f = d.shl[j];
      if constexpr (B) {
        T W[SH_DOF][4];
#pragma unroll
        for (int a = 0; a < SH_DOF; ++a) W[a][0] = W[a][1] = W[a][2] = W[a][3] = 0;
        for (int64_t i = d.foff[10][f]; i < d.foff[10][f + 1]; ++i) addW_rows<10, 1, T, CD, SH_DOF, 4>(d, i, W);
        pair_contrib<T, SH_DOF, 4>(d, f, W, acc, acc + NS);
      } else {
        for (int64_t i = d.foff[10][f]; i < d.foff[10][f + 1]; ++i) shape_a_rows<10, T, CD>(d, i, U, g);
      }
    }
  }
  T* o = block_sum_arr<T, K>(acc, lds);
  for (int k = threadIdx.x; k < K; k += blockDim.x) atomicAdd(d.shacc + (int64_t)SH_ACC * ch.x + k, (double)o[k]);
}

// pass A: U_ss, g_s and D_s of each shape from its accumulator
__global__ void k_shape_a_fin(Dev d) {
  constexpr int NS = SH_DOF * (SH_DOF + 1) / 2;
  const int q = blockIdx.x;
  const double* a = d.shacc + (int64_t)SH_ACC * q;
  const int e0 = a_grp(d, 3, q);
  for (int k = threadIdx.x; k < SH_DOF * SH_DOF; k += blockDim.x)
    d.Ush[(int64_t)SH_DOF * SH_DOF * q + k] = a[sym<SH_DOF>(k / SH_DOF, k % SH_DOF)];
  for (int k = threadIdx.x; k < SH_DOF; k += blockDim.x) {
    d.gA[e0 + k] = a[NS + k];
    d.DA[e0 + k] = fmin(fmax(a[sym<SH_DOF>(k, k)], 1e-6), 1e32);
  }
}

// pass B: the damped diagonal block of S and b of each shape
__global__ void k_shape_b_fin(Dev d, double lam) {
  constexpr int NS = SH_DOF * (SH_DOF + 1) / 2;
  const int q = blockIdx.x;
  const double* a = d.shacc + (int64_t)SH_ACC * q;
  const int e0 = a_grp(d, 3, q);
  for (int k = threadIdx.x; k < SH_DOF * SH_DOF; k += blockDim.x) {
    const int r = k / SH_DOF, c = k % SH_DOF;
    const int64_t idx = (int64_t)SH_DOF * SH_DOF * q + k;
    double v = d.Ush[idx] + a[sym<SH_DOF>(r, c)];
    if (r == c) v += lam * d.DA[e0 + r];
    d.Ssh[idx] = v;
  }
  for (int k = threadIdx.x; k < SH_DOF; k += blockDim.x) d.bA[e0 + k] = -d.gA[e0 + k] + a[NS + k];
}

void launch_shape_pass_a(const Dev& d, hipStream_t s) {
  if (!d.ns) return;
  launch_zero(d.shacc, (size_t)d.ns * SH_ACC * sizeof(double), s);
  if (d.n_shch) BA_DISPATCH_T_CD(d, k_shape_chunk<T, CD, false><<<d.n_shch, 256, 0, s>>>(d));
  k_shape_a_fin<<<d.ns, 128, 0, s>>>(d);
}

void launch_shape_pass_b(const Dev& d, double lambda, hipStream_t s) {
  if (!d.ns) return;
  launch_zero(d.shacc, (size_t)d.ns * SH_ACC * sizeof(double), s);
  if (d.n_shch) BA_DISPATCH_T_CD(d, k_shape_chunk<T, CD, true><<<d.n_shch, 256, 0, s>>>(d));
  k_shape_b_fin<<<d.ns, 128, 0, s>>>(d, lambda);
}

// S Z rows of the shapes: one workgroup per chunk, as k_sz_grp for a plane, the sums
// added to the shape's accumulator (d.shsz, cleared first); k_sz_shape_fin writes the rows
template <typename T, int CD, int L, int CPL>
__global__ __launch_bounds__(256) void k_sz_shape(Dev d, const T* Zr, const T* sfp, const T* sfl, double lam) {
  constexpr int R = 256 / L, NCOL = L * CPL;
  __shared__ double lds[4 * SH_DOF * NCOL];
  const int4 ch = d.shch[blockIdx.x];
  const int col = (threadIdx.x % L) * CPL, rs = threadIdx.x / L;
  const SzPanels P = sz_panels(d);
  const int pn = col / SZ_COLS, pc = col % SZ_COLS;
  const T* zr = Zr + pn * P.z + pc;
  const T* sp = sfp + pn * P.p + pc;
  const T* sl = sfl + pn * P.l + pc;
  double acc[SH_DOF][CPL];
#pragma unroll
  for (int k = 0; k < SH_DOF; ++k)
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[k][c] = 0;
  // every member of a chunk is on the chunk's shape (one shape per point or line)
  T zs[SH_DOF][CPL];
  z_cols<SH_DOF, CPL>(zr, a_grp(d, 3, ch.x), zs);
  for (int j = ch.y + rs; j < ch.y + ch.z; j += R) {
    if (ch.w == 0) {
      const int f = d.shp[j];
      for (int64_t i = d.foff[9][f]; i < d.foff[9][f + 1]; ++i)
        sz_shape_rec<9, 1, T, CD, CPL>(d, i, zs, zr, sp + (int64_t)f * 3 * SZ_COLS, acc);
    } else {
      const int f = d.shl[j];
      for (int64_t i = d.foff[10][f]; i < d.foff[10][f + 1]; ++i)
        sz_shape_rec<10, 1, T, CD, CPL>(d, i, zs, zr, sl + (int64_t)f * 4 * SZ_COLS, acc);
    }
  }
  double* out = d.shsz + (int64_t)SH_DOF * SZ_COLS * SZ_PANELS * ch.x;
  sz_block_sum<SH_DOF, L, CPL>(acc, lds, [&](int row, int cc, double v) {
    atomicAdd(out + row * SZ_COLS * SZ_PANELS + cc, v);
  });
}

__global__ void k_sz_shape_fin(Dev d, double lam) {
  const int q = blockIdx.x, e0 = a_grp(d, 3, q);
  const double* a = d.shsz + (int64_t)SH_DOF * SZ_COLS * SZ_PANELS * q;
  for (int t = threadIdx.x; t < SH_DOF * SZ_COLS * SZ_PANELS; t += blockDim.x) {
    const int row = t / (SZ_COLS * SZ_PANELS), cc = t % (SZ_COLS * SZ_PANELS);
    const int col = sz_col(cc / SZ_COLS, cc % SZ_COLS);
    if (col < 0 || col >= d.coarse_k) continue;
    const int e = e0 + row;
    d.SZc[(int64_t)col * d.nA + e] = a[t] + lam * d.DA[e] * d.Zc[(int64_t)col * d.nA + e];
  }
}

// x [+] h of every shape (the tangent updates of ba_shape.h), one thread per shape
__global__ void k_shape_retract(Dev d) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= d.ns) return;
  const double* P = d.sh64 + (int64_t)SH_STRIDE * q;
  double* o = d.sh64n + (int64_t)SH_STRIDE * q;
  const double* h = d.x + d.offSh + SH_DOF * q;
  for (int k = 0; k < SH_STRIDE; ++k) o[k] = P[k];
  const int type = shape_type(P);
  auto rot_right = [&](const double* w) {  // R' = R Exp(w), R row-major in P[0..8]
    double E[9];
    so3_exp(w, E);
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) o[3 * r + k] = P[3 * r] * E[k] + P[3 * r + 1] * E[3 + k] + P[3 * r + 2] * E[6 + k];
  };
  if (type == SH_SPHERE) {
    for (int k = 0; k < 3; ++k) o[k] = P[k] + h[k];
    o[3] = P[3] + h[3];
  } else if (type == SH_CYLINDER) {
    double E[9];
    so3_exp(h, E);
    // U' = U E with U = [u1 u2 u3] (columns stored consecutively), as for the lines
    for (int col = 0; col < 3; ++col)
      for (int r = 0; r < 3; ++r) o[3 * col + r] = P[r] * E[col] + P[3 + r] * E[3 + col] + P[6 + r] * E[6 + col];
    const double cph = cos(h[3]), sph = sin(h[3]);
    o[9] = P[9] * cph - P[10] * sph;
    o[10] = P[9] * sph + P[10] * cph;
    o[11] = P[11] + h[4];
  } else if (type == SH_CONE) {
    for (int k = 0; k < 3; ++k) o[k] = P[k] + h[k];
    s2_retract(P + 3, P + 6, P + 9, h[3], h[4], o + 3);
    s2_basis(o + 3, o + 6, o + 9);
    o[12] = P[12] + h[5];
  } else if (type == SH_ELLIPSOID) {
    rot_right(h);
    for (int k = 0; k < 3; ++k) {
      o[9 + k] = P[9 + k] + h[3 + k];
      o[12 + k] = P[12 + k] + h[6 + k];
    }
  } else {
    rot_right(h);
    for (int k = 0; k < 6; ++k) o[9 + k] = P[9 + k] + h[3 + k];
  }
}

// similarity-gauge rows of the shapes (rotation e_k about the origin, translation e_k,
// scale), the motion of each shape's tangent coordinates under the world motion that
// moves the cameras and groups of k_gauge_basis (one thread per shape)
__global__ void k_shape_gauge(Dev d) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= d.ns) return;
  const double* P = d.sh64 + (int64_t)SH_STRIDE * q;
  double g[SH_DOF][COARSE_GAUGE];
  for (int r = 0; r < SH_DOF; ++r)
    for (int c = 0; c < COARSE_GAUGE; ++c) g[r][c] = 0.0;
  const int type = shape_type(P);
  // a point c of the shape: e_k x c (rotation), e_k (translation), c (scale)
  auto point_rows = [&](int r0, const double* c) {
    for (int k = 0; k < 3; ++k) {
      double e[3] = {0, 0, 0}, ec[3];
      e[k] = 1.0;
      cross3(e, c, ec);
      for (int i = 0; i < 3; ++i) {
        g[r0 + i][k] = ec[i];
        g[r0 + i][3 + k] = e[i];
        g[r0 + i][6] = c[i];
      }
    }
  };
  if (type == SH_SPHERE) {
    point_rows(0, P);
    g[3][6] = 1.0;
  } else if (type == SH_CYLINDER) {
    const double *u1 = P, *u2 = P + 3, *u3 = P + 6, w1 = P[9], w2 = P[10];
    const double kap = w2 / w1, wn = w1 * w1 / (w1 * w1 + w2 * w2);
    for (int k = 0; k < 3; ++k) {
      // rotation: U <- Exp(e_k) U = U Exp(U^T e_k)
      g[0][k] = u1[k]; g[1][k] = u2[k]; g[2][k] = u3[k];
      // translation: the foot moves by e_k - (e_k . u1) u1
      g[0][3 + k] = fabs(kap) > 1e-12 ? -u2[k] / kap : 0.0;
      g[3][3 + k] = u3[k] * wn;
    }
    g[3][6] = kap * wn;  // scale: the foot (w2 / w1) u3 scales
    g[4][6] = 1.0;
  } else if (type == SH_CONE) {
    point_rows(0, P);
    const double* ax = P + 3;
    for (int k = 0; k < 3; ++k) {
      double e[3] = {0, 0, 0}, ea[3];
      e[k] = 1.0;
      cross3(e, ax, ea);
      g[3][k] = dot3(P + 6, ea);
      g[4][k] = dot3(P + 9, ea);
    }
  } else if (type == SH_ELLIPSOID) {
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < 3; ++i) g[i][k] = P[3 * k + i];  // R^T e_k
    point_rows(3, P + 9);
    for (int i = 0; i < 3; ++i) g[6 + i][6] = 1.0;
  } else {
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < 3; ++i) g[i][k] = P[3 * k + i];
    for (int f = 0; f < 6; ++f) {
      double n[3];
      cuboid_normal(P, f, n);
      for (int k = 0; k < 3; ++k) g[3 + f][3 + k] = -n[k];
      g[3 + f][6] = P[9 + f];
    }
  }
  const int e0 = a_grp(d, 3, q);
  for (int c = 0; c < COARSE_GAUGE; ++c)
    for (int r = 0; r < SH_DOF; ++r) d.Zc[(int64_t)c * d.nA + e0 + r] = g[r][c];
}

void launch_shape_gauge(const Dev& d, hipStream_t s) {
  if (d.ns) k_shape_gauge<<<nblk(d.ns, 64), 64, 0, s>>>(d);
}

}  // namespace ba
