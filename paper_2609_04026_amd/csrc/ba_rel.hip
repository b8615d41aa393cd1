// Inter-group relations (Sec. 3.2): orthogonality and parallelism between pairs of
// VPs and between pairs of plane normals.  Their records involve two groups of A and
// no camera or feature, so they only add to the group blocks of U and g (H_gg) and,
// through U, to the diagonal blocks of S and to the product S x.  They are few (pairs
// of groups), so everything here is FP64, one thread per record or per group block;
// each sum runs in a fixed order.
//
// Residuals of the unit directions u_a, u_b (the VP, or the plane normal):
//   orthogonal r = u_a . u_b (1 row), parallel r = u_a x u_b (3 rows); tangent
//   coordinates as for the groups themselves: a VP's 2, a plane's (dn, dw) with the
//   direction moving along b1, b2 and not with dw.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ba_internal.h"
#include "ba_math.h"

namespace ba {

namespace {

inline unsigned nblk_rel(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

constexpr int REL_COLS = 6;  // [J_a (3) | J_b (3)]

// sum over the 64 lanes of a wavefront (butterfly: every lane gets the same total)
__device__ __forceinline__ double rel_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ bool rel_plane(int kind) { return kind >= 2; }
__device__ __forceinline__ bool rel_parallel(int kind) { return kind == 1 || kind == 3; }
__device__ __forceinline__ int rel_rows(int kind) { return rel_parallel(kind) ? 3 : 1; }

// a relation whose group (either one) is left out by the record mask
__device__ __forceinline__ bool rel_masked(const Dev& d, int i) {
  if (!d.has_mask) return false;
  const uint8_t* m = rel_plane(d.rel_kind[i]) ? d.mpl : d.mvp;
  return m[d.rel_ga[i]] != 0 || m[d.rel_gb[i]] != 0;
}

// direction and tangent basis of group g of a relation kind, from the FP64 parameters
__device__ __forceinline__ void rel_dir(const Dev& d, int kind, int g, bool candidate, double (&u)[3], double (&b1)[3],
                                        double (&b2)[3]) {
  const double* p = rel_plane(kind) ? (candidate ? d.pl64n : d.pl64) + (int64_t)PL_STRIDE * g
                                    : (candidate ? d.vp64n : d.vp64) + (int64_t)VP_STRIDE * g;
#pragma unroll
  for (int i = 0; i < 3; ++i) { u[i] = p[i]; b1[i] = p[4 + i]; b2[i] = p[7 + i]; }
}

__device__ __forceinline__ void rel_residual(int kind, const double (&ua)[3], const double (&ub)[3], double (&r)[3]) {
  if (rel_parallel(kind)) {
    cross3(ua, ub, r);
  } else {
    r[0] = dot3(ua, ub);
    r[1] = r[2] = 0.0;
  }
}

// r~, J~ of every relation record
__global__ __launch_bounds__(256) void k_rel_lin(Dev d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n_rel) return;
  const int kind = d.rel_kind[i];
  double ua[3], a1[3], a2[3], ub[3], b1[3], b2[3];
  rel_dir(d, kind, d.rel_ga[i], false, ua, a1, a2);
  rel_dir(d, kind, d.rel_gb[i], false, ub, b1, b2);
  double r[3], J[3][REL_COLS];
  rel_residual(kind, ua, ub, r);
#pragma unroll
  for (int row = 0; row < 3; ++row)
#pragma unroll
    for (int c = 0; c < REL_COLS; ++c) J[row][c] = 0.0;
  const double* ta[2] = {a1, a2};
  const double* tb[2] = {b1, b2};
  for (int k = 0; k < 2; ++k) {
    if (rel_parallel(kind)) {
      double ca[3], cb[3];
      cross3(ta[k], ub, ca);  // d(u_a x u_b) along u_a's tangent k
      cross3(ua, tb[k], cb);
#pragma unroll
      for (int row = 0; row < 3; ++row) { J[row][k] = ca[row]; J[row][3 + k] = cb[row]; }
    } else {
      J[0][k] = dot3(ta[k], ub);
      J[0][3 + k] = dot3(ua, tb[k]);
    }
  }
  const double s = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  double rho, drho;
  loss_eval<double>(d.rel_lkind[kind], d.rel_lscale[kind], s, rho, drho);
  const double ws = rel_masked(d, i) ? 0.0 : sqrt(d.rel_lweight[kind] * drho);
#pragma unroll
  for (int row = 0; row < 3; ++row) {
    d.rel_r[3 * (int64_t)i + row] = ws * r[row];
#pragma unroll
    for (int c = 0; c < REL_COLS; ++c) d.rel_J[((int64_t)i * 3 + row) * REL_COLS + c] = ws * J[row][c];
  }
}

// group block b (planes, then VPs): its offset in A and its size
__device__ __forceinline__ void rel_block(const Dev& d, int b, int& o, int& n) {
  if (b < d.ng) { o = d.offPl + 3 * b; n = 3; }
  else { o = d.offVp + 2 * (b - d.ng); n = 2; }
}

// U_gg += J~_g^T J~_g, g_g += J~_g^T r~ over the block's relation entries, then its
// damping diagonal from the updated U (one thread per group block, after the group
// pass A has written the feature-record sums)
__global__ __launch_bounds__(256) void k_rel_a(Dev d) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= d.ng + d.nv) return;
  const int e0 = d.rel_goff[b], e1 = d.rel_goff[b + 1];
  if (e0 == e1) return;
  int o, n;
  rel_block(d, b, o, n);
  double U[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, g[3] = {0, 0, 0};
  for (int e = e0; e < e1; ++e) {
    const int ent = d.rel_gent[e], i = ent >> 1, c0 = 3 * (ent & 1);
    for (int row = 0; row < 3; ++row) {
      const double* Jr = d.rel_J + ((int64_t)i * 3 + row) * REL_COLS + c0;
      const double rr = d.rel_r[3 * (int64_t)i + row];
      for (int a = 0; a < n; ++a) {
        g[a] += Jr[a] * rr;
        for (int c = 0; c < n; ++c) U[a][c] += Jr[a] * Jr[c];
      }
    }
  }
  double* Ub = b < d.ng ? d.Upl + 9 * b : d.Uvp + 4 * (b - d.ng);
  for (int a = 0; a < n; ++a) {
    for (int c = 0; c < n; ++c) Ub[a * n + c] += U[a][c];
    d.gA[o + a] += g[a];
    d.DA[o + a] = fmin(fmax(Ub[a * n + a], 1e-6), 1e32);
  }
}

// rel_y, group rows: sum over the block's entries of J~_side^T (J~_a x_a + J~_b x_b)
template <typename T> __global__ __launch_bounds__(256) void k_rel_mv(Dev d, const double* done) {
  if (done && *done != 0.0) return;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= d.ng + d.nv) return;
  const T* x = (const T*)d.xT;
  int o, n;
  rel_block(d, b, o, n);
  const bool plane = b < d.ng;
  double y[3] = {0, 0, 0};
  for (int e = d.rel_goff[b]; e < d.rel_goff[b + 1]; ++e) {
    const int ent = d.rel_gent[e], i = ent >> 1, c0 = 3 * (ent & 1);
    const int oa = plane ? d.offPl + 3 * d.rel_ga[i] : d.offVp + 2 * d.rel_ga[i];
    const int ob = plane ? d.offPl + 3 * d.rel_gb[i] : d.offVp + 2 * d.rel_gb[i];
    for (int row = 0; row < 3; ++row) {
      const double* Jr = d.rel_J + ((int64_t)i * 3 + row) * REL_COLS;
      double t = 0;
      for (int a = 0; a < n; ++a) t += Jr[a] * (double)x[oa + a] + Jr[3 + a] * (double)x[ob + a];
      for (int a = 0; a < n; ++a) y[a] += Jr[c0 + a] * t;
    }
  }
  for (int a = 0; a < n; ++a) d.rel_y[o + a] = y[a];
}

// S Z += U_rel Z in the group rows of every active coarse column (one thread per group
// block and column; Z and S Z are FP64, column-major)
__global__ __launch_bounds__(256) void k_rel_sz(Dev d) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nb = d.ng + d.nv;
  if (t >= nb * d.coarse_k) return;
  const int b = t % nb, col = t / nb;
  int o, n;
  rel_block(d, b, o, n);
  const bool plane = b < d.ng;
  const double* z = d.Zc + (int64_t)col * d.nA;
  double y[3] = {0, 0, 0};
  for (int e = d.rel_goff[b]; e < d.rel_goff[b + 1]; ++e) {
    const int ent = d.rel_gent[e], i = ent >> 1, c0 = 3 * (ent & 1);
    const int oa = plane ? d.offPl + 3 * d.rel_ga[i] : d.offVp + 2 * d.rel_ga[i];
    const int ob = plane ? d.offPl + 3 * d.rel_gb[i] : d.offVp + 2 * d.rel_gb[i];
    for (int row = 0; row < 3; ++row) {
      const double* Jr = d.rel_J + ((int64_t)i * 3 + row) * REL_COLS;
      double u = 0;
      for (int a = 0; a < n; ++a) u += Jr[a] * z[oa + a] + Jr[3 + a] * z[ob + a];
      for (int a = 0; a < n; ++a) y[a] += Jr[c0 + a] * u;
    }
  }
  double* sz = d.SZc + (int64_t)col * d.nA;
  for (int a = 0; a < n; ++a) sz[o + a] += y[a];
}

// FP64 cost of the relations at the current or candidate parameters: one partial
__global__ __launch_bounds__(256) void k_rel_cost(Dev d, int candidate, double* part) {
  __shared__ double lds[5];
  double e = 0;
  for (int i = threadIdx.x; i < d.n_rel; i += blockDim.x) {
    if (rel_masked(d, i)) continue;
    const int kind = d.rel_kind[i];
    double ua[3], a1[3], a2[3], ub[3], b1[3], b2[3], r[3];
    rel_dir(d, kind, d.rel_ga[i], candidate != 0, ua, a1, a2);
    rel_dir(d, kind, d.rel_gb[i], candidate != 0, ub, b1, b2);
    rel_residual(kind, ua, ub, r);
    double rho, drho;
    loss_eval<double>(d.rel_lkind[kind], d.rel_lscale[kind], r[0] * r[0] + r[1] * r[1] + r[2] * r[2], rho, drho);
    e += 0.5 * d.rel_lweight[kind] * rho;
  }
  e = rel_wave_sum(e);  // fixed-order workgroup sum
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += lds[k];
    part[0] = t;
  }
}

// model decrease: + sum over the relations of |J~ h_a|^2 (h_a = d.x), added to SC_JH2
// after the feature records' sum has been written there
__global__ __launch_bounds__(256) void k_rel_md(Dev d) {
  __shared__ double lds[5];
  double acc = 0;
  for (int i = threadIdx.x; i < d.n_rel; i += blockDim.x) {
    const bool plane = d.rel_kind[i] >= 2;
    const int n = plane ? 3 : 2;
    const int oa = plane ? d.offPl + 3 * d.rel_ga[i] : d.offVp + 2 * d.rel_ga[i];
    const int ob = plane ? d.offPl + 3 * d.rel_gb[i] : d.offVp + 2 * d.rel_gb[i];
    for (int row = 0; row < 3; ++row) {
      const double* Jr = d.rel_J + ((int64_t)i * 3 + row) * REL_COLS;
      double t = 0;
      for (int a = 0; a < n; ++a) t += Jr[a] * d.x[oa + a] + Jr[3 + a] * d.x[ob + a];
      acc += t * t;
    }
  }
  acc = rel_wave_sum(acc);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += lds[k];
    d.scal[SC_JH2] += t;
  }
}

}  // namespace

void launch_rel_linearize(const Dev& d, hipStream_t s) {
  if (d.n_rel) k_rel_lin<<<nblk_rel(d.n_rel, 256), 256, 0, s>>>(d);
}

void launch_rel_a(const Dev& d, hipStream_t s) {
  if (d.n_rel && d.ng + d.nv) k_rel_a<<<nblk_rel(d.ng + d.nv, 256), 256, 0, s>>>(d);
}

void launch_rel_matvec(const Dev& d, const double* done, hipStream_t s) {
  if (!d.n_rel || !(d.ng + d.nv)) return;
  if (d.fp64) k_rel_mv<double><<<nblk_rel(d.ng + d.nv, 256), 256, 0, s>>>(d, done);
  else k_rel_mv<float><<<nblk_rel(d.ng + d.nv, 256), 256, 0, s>>>(d, done);
}

void launch_rel_sz(const Dev& d, hipStream_t s) {
  if (d.n_rel && d.coarse_k > 0 && d.ng + d.nv)
    k_rel_sz<<<nblk_rel((int64_t)(d.ng + d.nv) * d.coarse_k, 256), 256, 0, s>>>(d);
}

void launch_rel_cost(const Dev& d, bool candidate, double* part, hipStream_t s) {
  if (d.n_rel) k_rel_cost<<<1, 256, 0, s>>>(d, candidate ? 1 : 0, part);
}

void launch_rel_md(const Dev& d, hipStream_t s) {
  if (d.n_rel) k_rel_md<<<1, 256, 0, s>>>(d);
}

}  // namespace ba
