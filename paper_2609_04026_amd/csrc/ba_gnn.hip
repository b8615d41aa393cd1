// Learned coarse-space correction of the reduced-system preconditioner.
//
// A message-passing network over the block graph of the reduced system
// (nodes: camera / plane / VP blocks; edges: blocks sharing a feature)
// predicts K = COARSE_K vectors per block, Y_i (n_i x K).  With unit row
// scales u_i, Z_i = diag(u_i) Y_i, and the PCG preconditioner becomes
//   P r = M r + Z E^-1 Z^T r,   M = blockdiag(S_ii)^-1,   E = Z^T S Z.
// Network (hidden width H = 64, gelu(x) = x/2 (1 + tanh(sqrt(2/pi)(x + 0.044715 x^3)))):
//   h = gelu(x W_in + b_in)
//   3 times:  m_i = mean_{edges j -> i} gelu([h_j, e_ji] W_e + b_e)
//             (computed as (h W_h)_j + e_ji W_x + b_e: the h-part per node, then one
//             pass over the edges)
//             h = gelu(h W_s + b_s + m) + h
//   Y_i = h_i W_t + b_t for the node's type t (row-major n_t x K)
// Training loss per system: tr((Z^T D Z)^-1 Z^T S Z), D = blockdiag(S_ii)
// (the sum of the Ritz values of the block-normalised system on span Z);
// a batch takes the mean over its systems.
//
// Dense layers are GEMMs on BF16 operands with FP32 accumulation
// (v_mfma_f32_16x16x16_bf16), or FP32 FMA in the debug precision; the
// message aggregation is a CSR mean; gradients accumulate in FP32; the
// block products of the loss and the coarse basis are FP64.
#include "ba_gnn.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <stdexcept>

#include "../../include/ba.h"

namespace {

using ba_gnn_impl::NODE_IN;
using ba_gnn_impl::EDGE_IN;
constexpr int H = 64, NIN = NODE_IN, EIN = EDGE_IN, EK = H + EIN, LAYERS = 3, HEADP = ba_gnn_impl::HEAD_PAD;
constexpr int KC = ba::COARSE_NET;    // network columns
constexpr int KG = ba::COARSE_GAUGE;  // gauge columns, first in the coarse basis
constexpr int KT = ba::COARSE_K;      // all columns
static_assert(HEADP == 9 * KC, "head rows are padded to 9 block rows of K entries");

struct Layout {
  size_t W_in = 0, b_in = 0, W_e[LAYERS] = {}, b_e[LAYERS] = {}, W_s[LAYERS] = {}, b_s[LAYERS] = {};
  size_t W_t[3] = {}, b_t[3] = {}, total = 0;
  int T[3] = {}, nb[3] = {};
};

Layout make_layout(int cd) {
  Layout L;
  size_t o = 0;
  L.W_in = o; o += (size_t)NIN * H;
  L.b_in = o; o += H;
  for (int l = 0; l < LAYERS; ++l) {
    L.W_e[l] = o; o += (size_t)EK * H;
    L.b_e[l] = o; o += H;
    L.W_s[l] = o; o += (size_t)H * H;
    L.b_s[l] = o; o += H;
  }
  L.nb[0] = cd; L.nb[1] = 3; L.nb[2] = 2;
  for (int t = 0; t < 3; ++t) {
    L.T[t] = L.nb[t] * KC;
    L.W_t[t] = o; o += (size_t)H * L.T[t];
    L.b_t[t] = o; o += L.T[t];
  }
  L.total = o;
  return L;
}

#define GCHK(call)                                                                              \
  do {                                                                                          \
    hipError_t _e = (call);                                                                     \
    if (_e != hipSuccess) throw std::runtime_error(std::string(#call) + ": " + hipGetErrorString(_e)); \
  } while (0)

unsigned nblk(int64_t n, int b) { return (unsigned)std::max<int64_t>(1, (n + b - 1) / b); }

// ---------------------------------------------------------------------------
// device helpers
__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// (1 + tanh(y)) / 2 is the logistic function of 2y, so gelu(x) = x / (1 + e^(-2y)) and
// gelu'(x) = s + 2 x s (1 - s) y'(x) with s = 1 / (1 + e^(-2y)): one hardware exp2 and one
// reciprocal per value (e^(-2y) overflows to inf for large negative x, giving s = 0)
__device__ __forceinline__ float gelu_s(float x) {
  const float c = 0.7978845608028654f, k = -2.0f * 1.4426950408889634f;  // -2 log2(e)
  const float y = c * (x + 0.044715f * x * x * x);
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(k * y));
}
__device__ __forceinline__ float gelu(float x) { return x * gelu_s(x); }
__device__ __forceinline__ float gelu_d(float x) {
  const float c = 0.7978845608028654f, s = gelu_s(x);
  return s + 2.0f * x * s * (1.0f - s) * c * (1.0f + 3.0f * 0.044715f * x * x);
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// operand view: element (i, j) at p[i * s0 + j * s1]
struct View {
  const void* p;
  int64_t s0, s1;
};

// C (M x N, ldc) [+]= A (M x K) B (K x N); one 16 x 16 output tile per wavefront,
// K split into `ksplit` ranges (then FP32 atomics into C)
template <bool BF16>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, View A, View B, float* C, int ldc, int ksplit,
                                              int mode /*0 store, 1 accumulate, 2 atomic*/) {
  const int wave = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const int tiles_m = (M + 15) / 16, tiles_n = (N + 15) / 16, ntile = tiles_m * tiles_n;
  if (wave >= ntile * ksplit) return;
  const int tile = wave % ntile, ks = wave / ntile;
  const int tm = tile / tiles_n, tn = tile % tiles_n;
  const int kchunk = ((K + ksplit - 1) / ksplit + 15) / 16 * 16;
  const int kb = ks * kchunk, ke = min(K, kb + kchunk);
  const int r = lane & 15, g = lane >> 4;
  float acc[4] = {0, 0, 0, 0};
  if constexpr (BF16) {
    const uint16_t* Ap = (const uint16_t*)A.p;
    const uint16_t* Bp = (const uint16_t*)B.p;
    f32x4 c = {0, 0, 0, 0};
    const int arow = tm * 16 + r, bcol = tn * 16 + r;
    for (int k0 = kb; k0 < ke; k0 += 16) {
      bf16x4 a, b;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + 4 * g + j;
        a[j] = (arow < M && k < ke) ? (short)Ap[arow * A.s0 + k * A.s1] : (short)0;
        b[j] = (bcol < N && k < ke) ? (short)Bp[k * B.s0 + bcol * B.s1] : (short)0;
      }
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = c[j];
  } else {
    const float* Ap = (const float*)A.p;
    const float* Bp = (const float*)B.p;
    const int col = tn * 16 + r;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = tm * 16 + 4 * g + j;
      float s = 0;
      if (row < M && col < N)
        for (int k = kb; k < ke; ++k) s += Ap[row * A.s0 + k * A.s1] * Bp[k * B.s0 + col * B.s1];
      acc[j] = s;
    }
  }
  const int col = tn * 16 + r;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = tm * 16 + 4 * g + j;
    if (row < M && col < N) {
      float* cp = C + (int64_t)row * ldc + col;
      if (mode == 2) atomicAdd(cp, acc[j]);
      else if (mode == 1) *cp += acc[j];
      else *cp = acc[j];
    }
  }
}

__global__ void k_cast_bf16(const float* src, uint16_t* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = f2bf(src[i]);
}

// z = Z + bias (+ extra); Z <- z; out = gelu(z) (+ resid)
__global__ void k_bias_act(float* Z, const float* bias, const float* extra, const float* resid, float* out, int rows, int cols) {
  const int64_t n = (int64_t)rows * cols;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float z = Z[i] + bias[i % cols];
    if (extra) z += extra[i];
    Z[i] = z;
    out[i] = gelu(z) + (resid ? resid[i] : 0.0f);
  }
}

__global__ void k_fill2d(float* C, int rows, int cols, int ld) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)rows * cols; i += (int64_t)gridDim.x * blockDim.x)
    C[(i / cols) * ld + i % cols] = 0.0f;
}

__global__ void k_bias_add(float* Z, const float* bias, int rows, int cols, int ld) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)rows * cols; i += (int64_t)gridDim.x * blockDim.x)
    Z[(i / cols) * ld + i % cols] += bias[i % cols];
}

__global__ void k_act_bwd(const float* dOut, const float* Zpre, float* dZ, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dZ[i] = dOut[i] * gelu_d(Zpre[i]);
}

// messages of one layer, with [h_j, e_ji] W_e = (h W_h)_j + e_ji W_x:
// Ze_e = Ph[src_e] + e_e W_x + b_e (stored when Ze != null), m_i = mean over in-edges of gelu(Ze).
// Work items are runs of <= EDGE_RUN in-edges of one node (high-degree nodes split
// over several items); one wavefront per run, one lane per channel, adding its run's
// share to Mm (cleared before) with FP32 atomics.  The run's source ids and edge inputs
// are loaded one edge per lane, and each edge's values are then read from its lane into
// scalar registers (v_readlane: the edge is the same on every lane), so that the only
// per-edge vector load is the 256-byte row Ph[src].
constexpr int EDGE_RUN = 32;
__device__ __forceinline__ float lane_f(float v, int k) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k)); }

__global__ void k_edge_msg(const float* Ph, const float* ex, const float* Wx, const float* be, const int32_t* src,
                           const int32_t* off, const int2* runs, int n_runs, float* Ze, float* Mm) {
  static_assert(EIN == 8, "edge inputs are read as two float4");
  static_assert(H == 64 && EDGE_RUN <= 64, "one wavefront per run, one lane per channel");
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)n_runs * H; i += (int64_t)gridDim.x * blockDim.x) {
    const int2 run = runs[i / H];  // (node, first edge)
    const int c = (int)(i % H), node = run.x;
    const int e0 = run.y, ne = min(off[node + 1], e0 + EDGE_RUN) - e0;
    float w[EIN];
#pragma unroll
    for (int k = 0; k < EIN; ++k) w[k] = Wx[k * H + c];
    const float bc = be[c];
    int my_src = 0;
    float4 x0 = make_float4(0, 0, 0, 0), x1 = x0;
    if (c < ne) {
      my_src = src[e0 + c];
      x0 = reinterpret_cast<const float4*>(ex)[2 * (int64_t)(e0 + c)];
      x1 = reinterpret_cast<const float4*>(ex)[2 * (int64_t)(e0 + c) + 1];
    }
    float acc = 0;
    auto edge = [&](int k, float p) {
      const float z = p + bc + lane_f(x0.x, k) * w[0] + lane_f(x0.y, k) * w[1] + lane_f(x0.z, k) * w[2] +
                      lane_f(x0.w, k) * w[3] + lane_f(x1.x, k) * w[4] + lane_f(x1.y, k) * w[5] +
                      lane_f(x1.z, k) * w[6] + lane_f(x1.w, k) * w[7];
      if (Ze) Ze[(int64_t)(e0 + k) * H + c] = z;
      acc += gelu(z);
    };
    int k = 0;
    for (; k + 4 <= ne; k += 4) {  // four rows of Ph in flight
      const float p0 = Ph[(int64_t)__builtin_amdgcn_readlane(my_src, k) * H + c];
      const float p1 = Ph[(int64_t)__builtin_amdgcn_readlane(my_src, k + 1) * H + c];
      const float p2 = Ph[(int64_t)__builtin_amdgcn_readlane(my_src, k + 2) * H + c];
      const float p3 = Ph[(int64_t)__builtin_amdgcn_readlane(my_src, k + 3) * H + c];
      edge(k, p0); edge(k + 1, p1); edge(k + 2, p2); edge(k + 3, p3);
    }
    for (; k < ne; ++k) edge(k, Ph[(int64_t)__builtin_amdgcn_readlane(my_src, k) * H + c]);
    atomicAdd(Mm + (int64_t)node * H + c, acc / (float)(off[node + 1] - off[node]));
  }
}

// The same pass for the attached problem graph, whose edge inputs are log1p(shared
// records) and a one-hot kind (columns 1-4; columns 5-7 zero): e W_x + b_e =
// e_0 W_x[0] + (W_x[kind] + b_e), so each edge takes its two words (value, kind) from its
// lane and the lane's four kind rows are selected instead of eight products.
__global__ void k_edge_msg_typed(const float* Ph, const int2* et, const float* Wx, const float* be, const int32_t* src,
                                 const int32_t* off, const int2* runs, int n_runs, float* Mm) {
  static_assert(H == 64 && EDGE_RUN <= 64, "one wavefront per run, one lane per channel");
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)n_runs * H; i += (int64_t)gridDim.x * blockDim.x) {
    const int2 run = runs[i / H];  // (node, first edge)
    const int c = (int)(i % H), node = run.x;
    const int e0 = run.y, ne = min(off[node + 1], e0 + EDGE_RUN) - e0;
    const float w0 = Wx[c], bc = be[c];
    const float t1 = Wx[H + c] + bc, t2 = Wx[2 * H + c] + bc, t3 = Wx[3 * H + c] + bc, t4 = Wx[4 * H + c] + bc;
    int my_src = 0;
    int2 my_e = make_int2(0, 1);
    if (c < ne) {
      my_src = src[e0 + c];
      my_e = et[e0 + c];
    }
    float acc = 0;
    auto edge = [&](int k, float p) {
      const float x0 = __int_as_float(__builtin_amdgcn_readlane(my_e.x, k));
      const int kind = __builtin_amdgcn_readlane(my_e.y, k);
      const float tk = kind == 1 ? t1 : kind == 2 ? t2 : kind == 3 ? t3 : t4;
      acc += gelu(p + x0 * w0 + tk);
    };
    int k = 0;
    for (; k + 4 <= ne; k += 4) {  // four rows of Ph in flight
      const float p0 = Ph[(int64_t)__builtin_amdgcn_readlane(my_src, k) * H + c];
      const float p1 = Ph[(int64_t)__builtin_amdgcn_readlane(my_src, k + 1) * H + c];
      const float p2 = Ph[(int64_t)__builtin_amdgcn_readlane(my_src, k + 2) * H + c];
      const float p3 = Ph[(int64_t)__builtin_amdgcn_readlane(my_src, k + 3) * H + c];
      edge(k, p0); edge(k + 1, p1); edge(k + 2, p2); edge(k + 3, p3);
    }
    for (; k < ne; ++k) edge(k, Ph[(int64_t)__builtin_amdgcn_readlane(my_src, k) * H + c]);
    atomicAdd(Mm + (int64_t)node * H + c, acc / (float)(off[node + 1] - off[node]));
  }
}

// dZe_e = dM[dst_e] / deg(dst_e) * gelu'(Ze_e)   (one thread per edge entry)
__global__ void k_edge_msg_bwd(const float* dM, const float* Ze, const int32_t* dst, const int32_t* off, float* dZe, int m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)m * H; i += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(i / H), c = (int)(i % H);
    const int d = dst[e];
    dZe[i] = dM[(int64_t)d * H + c] / (float)(off[d + 1] - off[d]) * gelu_d(Ze[i]);
  }
}

// dP_j = sum over edges out of j of dZe (the reverses of the edges into j), stride H
__global__ void k_scatter_src(const float* dZe, const int32_t* rev, const int32_t* off, float* dP, int n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)n * H; i += (int64_t)gridDim.x * blockDim.x) {
    const int node = (int)(i / H), c = (int)(i % H);
    float s = 0;
    for (int k = off[node]; k < off[node + 1]; ++k) s += dZe[(int64_t)rev[k] * H + c];
    dP[i] = s;
  }
}

__global__ void k_colsum(const float* X, int rows, int cols, int ld, float* out) {
  // blockDim = 256: 4 groups of 64 columns chunks
  const int c = blockIdx.y * 64 + (threadIdx.x & 63);
  const int part = threadIdx.x >> 6;
  if (c >= cols) return;
  float s = 0;
  for (int r = blockIdx.x * 4 + part; r < rows; r += gridDim.x * 4) s += X[(int64_t)r * ld + c];
  atomicAdd(out + c, s);
}

__global__ void k_add(float* a, const float* b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] += b[i];
}

__device__ __forceinline__ int node_size(int type, int cd) { return type == 0 ? cd : type == 1 ? 3 : 2; }

// entry (row r, column c) of the coarse basis of node j: gauge columns first, then
// the network's head scaled by the row's unit
__device__ __forceinline__ double zval(const float* heads, const float* unit, const double* gauge, int j, int r, int c) {
  if (c < KG) return gauge[((int64_t)j * 9 + r) * KG + c];
  return (double)unit[(int64_t)j * 9 + r] * (double)heads[(int64_t)j * HEADP + r * KC + (c - KG)];
}

// SZ_i = S_ii Z_i + sum_{edges j -> i} S_ij Z_j and DZ_i = S_ii Z_i (FP64, n x 9 x KT),
// one thread per (node, row, column)
__global__ void k_coarse_products(const float* heads, const float* unit, const double* gauge, const int32_t* type,
                                  const int32_t* src, const int32_t* dst_off, const double* s_node,
                                  const int64_t* s_node_off, const double* s_edge, const int64_t* s_edge_off, int n,
                                  int cd, double* SZ, double* DZ) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * 9 * KT) return;
  const int i = (int)(t / (9 * KT)), r = (int)(t % (9 * KT)) / KT, c = (int)(t % KT);
  const int ni = node_size(type[i], cd);
  if (r >= ni) { SZ[t] = 0; DZ[t] = 0; return; }
  const double* Sii = s_node + s_node_off[i] + (int64_t)r * ni;
  double dz = 0;
  for (int q = 0; q < ni; ++q) dz += Sii[q] * zval(heads, unit, gauge, i, q, c);
  double sz = dz;
  for (int e = dst_off[i]; e < dst_off[i + 1]; ++e) {
    const int j = src[e];
    const int nj = node_size(type[j], cd);
    const double* Se = s_edge + s_edge_off[e] + (int64_t)r * nj;
    for (int q = 0; q < nj; ++q) sz += Se[q] * zval(heads, unit, gauge, j, q, c);
  }
  SZ[t] = sz;
  DZ[t] = dz;
}

// per-system Gram matrices A = Z^T S Z and G = Z^T D Z (KT x KT, FP64 atomics),
// one thread per (node, a, b)
__global__ void k_coarse_gram(const float* heads, const float* unit, const double* gauge, const int32_t* type,
                              const int32_t* graph, const double* SZ, const double* DZ, int n, int cd, double* Ag,
                              double* Gg) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * KT * KT) return;
  const int i = (int)(t / (KT * KT)), a = (int)(t % (KT * KT)) / KT, b = (int)(t % KT);
  const int ni = node_size(type[i], cd);
  double sa = 0, sg = 0;
  for (int r = 0; r < ni; ++r) {
    const double z = zval(heads, unit, gauge, i, r, a);
    sa += z * SZ[((int64_t)i * 9 + r) * KT + b];
    sg += z * DZ[((int64_t)i * 9 + r) * KT + b];
  }
  const int64_t o = (int64_t)graph[i] * KT * KT + a * KT + b;
  atomicAdd(Ag + o, sa);
  atomicAdd(Gg + o, sg);
}

// per system: loss tr(G^-1 A) / n_graphs, Q1 = G^-1, Q2 = G^-1 A G^-1 (A symmetrised);
// a system whose G is not positive definite adds nothing (Q1 = Q2 = 0) and is counted
__global__ void k_coarse_loss(const double* Ag, const double* Gg, int n_graphs, double* Q1, double* Q2, double* loss,
                              double* n_bad) {
  const int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= n_graphs) return;
  const double* A = Ag + (int64_t)gi * KT * KT;
  const double* G = Gg + (int64_t)gi * KT * KT;
  double L[KT][KT], X[KT][KT], Gi[KT][KT], As[KT][KT];
  bool ok = true;
  for (int p = 0; p < KT; ++p)
    for (int q = 0; q < KT; ++q) {
      L[p][q] = 0.5 * (G[p * KT + q] + G[q * KT + p]);
      As[p][q] = 0.5 * (A[p * KT + q] + A[q * KT + p]);
      X[p][q] = 0.0;
    }
  for (int j = 0; j < KT && ok; ++j) {
    double s = L[j][j];
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    if (!(s > 0.0) || !isfinite(s)) { ok = false; break; }
    const double ljj = sqrt(s);
    L[j][j] = ljj;
    for (int r = j + 1; r < KT; ++r) {
      double u = L[r][j];
      for (int k = 0; k < j; ++k) u -= L[r][k] * L[j][k];
      L[r][j] = u / ljj;
    }
  }
  double* q1 = Q1 + (int64_t)gi * KT * KT;
  double* q2 = Q2 + (int64_t)gi * KT * KT;
  if (!ok) {
    for (int k = 0; k < KT * KT; ++k) { q1[k] = 0; q2[k] = 0; }
    atomicAdd(n_bad, 1.0);
    return;
  }
  for (int c = 0; c < KT; ++c)  // X = L^-1
    for (int r = c; r < KT; ++r) {
      double s = r == c ? 1.0 : 0.0;
      for (int k = c; k < r; ++k) s -= L[r][k] * X[k][c];
      X[r][c] = s / L[r][r];
    }
  for (int p = 0; p < KT; ++p)  // G^-1 = X^T X
    for (int q = 0; q < KT; ++q) {
      double s = 0;
      for (int k = 0; k < KT; ++k) s += X[k][p] * X[k][q];
      Gi[p][q] = s;
    }
  double tr = 0;
  for (int p = 0; p < KT; ++p)
    for (int q = 0; q < KT; ++q) tr += Gi[p][q] * As[q][p];
  for (int p = 0; p < KT; ++p)  // L <- G^-1 A (reusing the storage)
    for (int q = 0; q < KT; ++q) {
      double s = 0;
      for (int k = 0; k < KT; ++k) s += Gi[p][k] * As[k][q];
      L[p][q] = s;
    }
  for (int p = 0; p < KT; ++p)
    for (int q = 0; q < KT; ++q) {
      double s = 0;
      for (int k = 0; k < KT; ++k) s += L[p][k] * Gi[k][q];
      q1[p * KT + q] = Gi[p][q];
      q2[p * KT + q] = s;
    }
  atomicAdd(loss, tr / n_graphs);
}

// d loss / d heads for the network columns: dZ = (2 / n_graphs) (SZ Q1 - DZ Q2), dY = u dZ
__global__ void k_coarse_dheads(const double* SZ, const double* DZ, const double* Q1, const double* Q2,
                                const float* unit, const int32_t* type, const int32_t* graph, int n, int cd,
                                int n_graphs, float* dheads) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * HEADP) return;
  const int i = (int)(t / HEADP), r = (int)(t % HEADP) / KC, c = KG + (int)(t % KC);
  if (r >= node_size(type[i], cd)) { dheads[t] = 0.0f; return; }
  const double* q1 = Q1 + (int64_t)graph[i] * KT * KT;
  const double* q2 = Q2 + (int64_t)graph[i] * KT * KT;
  const double* sz = SZ + ((int64_t)i * 9 + r) * KT;
  const double* dz = DZ + ((int64_t)i * 9 + r) * KT;
  double s = 0;
  for (int b = 0; b < KT; ++b) s += sz[b] * q1[b * KT + c] - dz[b] * q2[b * KT + c];
  dheads[t] = (float)(2.0 / n_graphs * s * unit[(int64_t)i * 9 + r]);
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1 - b1) * gi;
    const float vi = b2 * v[i] + (1 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// ---------------------------------------------------------------------------
// node input features from the damped diagonal blocks of S, the structural
// entries and the current geometry
__global__ void k_node_features(ba::Dev d, const float* stat, const int32_t* type, int n, double lam, double s0,
                                float* X) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t = type[i];
  int nb;
  const double* S;
  if (t == 0) { nb = d.CD; S = d.Scam + (int64_t)d.CD * d.CD * i; }
  else if (t == 1) { nb = 3; S = d.Spl + 9 * (int64_t)(i - d.nc); }
  else { nb = 2; S = d.Svp + 4 * (int64_t)(i - d.nc - d.ng); }
  float* x = X + (int64_t)i * NIN;
  for (int k = 0; k < NIN; ++k) x[k] = stat[(int64_t)i * NIN + k];
  // log of the diagonal in unit-scaled coordinates (u_p^2 S_pp), centred
  double ld[9], mean = 0;
  for (int k = 0; k < nb; ++k) {
    const bool len = (t == 0 && k >= 3 && k < 6) || (t == 1 && k == 2);
    ld[k] = log(fmax(S[k * nb + k], 1e-300)) + (len ? 2.0 * log(s0) : 0.0);
    mean += ld[k];
  }
  mean /= nb;
  for (int k = 0; k < nb; ++k) x[k] = (float)(ld[k] - mean);
  int c = 9;
  for (int p = 1; p < nb; ++p)
    for (int q = 0; q < p; ++q, ++c) x[c] = (float)(S[p * nb + q] / sqrt(fmax(S[p * nb + p] * S[q * nb + q], 1e-300)));
  x[45] = (float)log(fmax(lam, 1e-300));
  if (t == 0) {  // R row-major, t / s0
    const double* cam = d.cam64 + (int64_t)ba::CAM_STRIDE * i;
    for (int k = 0; k < 9; ++k) x[51 + k] = (float)cam[k];
    for (int k = 0; k < 3; ++k) x[60 + k] = (float)(cam[9 + k] / s0);
  } else if (t == 1) {  // n, w / s0, b1, b2
    const double* pl = d.pl64 + (int64_t)ba::PL_STRIDE * (i - d.nc);
    for (int k = 0; k < 3; ++k) x[51 + k] = (float)pl[k];
    x[54] = (float)(pl[3] / s0);
    for (int k = 0; k < 6; ++k) x[55 + k] = (float)pl[4 + k];
  } else {  // v, b1, b2
    const double* vp = d.vp64 + (int64_t)ba::VP_STRIDE * (i - d.nc - d.ng);
    for (int k = 0; k < 3; ++k) x[51 + k] = (float)vp[k];
    for (int k = 0; k < 6; ++k) x[54 + k] = (float)vp[4 + k];
  }
}

// the network's columns of Z (after the gauge columns; column-major, FP64) from the heads
__global__ void k_coarse_basis(ba::Dev d, const float* heads, const int32_t* type, int n, double s0) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * HEADP) return;
  const int i = (int)(t / HEADP), r = (int)(t % HEADP) / KC, c = (int)(t % KC);
  const int ty = type[i];
  const int nb = node_size(ty, d.CD);
  if (r >= nb) return;
  int o;
  double u = 1.0;
  if (ty == 0) { o = d.CD * i; if (r >= 3 && r < 6) u = s0; }
  else if (ty == 1) { o = d.offPl + 3 * (i - d.nc); if (r == 2) u = s0; }
  else { o = d.offVp + 2 * (i - d.nc - d.ng); }
  d.Zc[(int64_t)(KG + c) * d.nA + o + r] = u * (double)heads[(int64_t)i * HEADP + r * KC + c];
}

// y = L^-1 v blockwise (inverse = false) or L^-T v (inverse = true), S_ii = L_i L_i^T
__global__ void k_block_tri(ba::Dev d, const double* v, double* y, int transposed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nbk = d.nc + d.ng + d.nv;
  if (i >= nbk) return;
  int nb, o;
  const double* S;
  if (i < d.nc) { nb = d.CD; S = d.Scam + (int64_t)d.CD * d.CD * i; o = d.CD * i; }
  else if (i < d.nc + d.ng) { nb = 3; S = d.Spl + 9 * (int64_t)(i - d.nc); o = d.offPl + 3 * (i - d.nc); }
  else { nb = 2; S = d.Svp + 4 * (int64_t)(i - d.nc - d.ng); o = d.offVp + 2 * (i - d.nc - d.ng); }
  double L[9][9];
  for (int p = 0; p < nb; ++p)
    for (int q = 0; q < nb; ++q) L[p][q] = 0.5 * (S[p * nb + q] + S[q * nb + p]);
  for (int j = 0; j < nb; ++j) {
    double s = L[j][j];
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    const double ljj = sqrt(fmax(s, 1e-300));
    L[j][j] = ljj;
    for (int r = j + 1; r < nb; ++r) {
      double u = L[r][j];
      for (int k = 0; k < j; ++k) u -= L[r][k] * L[j][k];
      L[r][j] = u / ljj;
    }
  }
  double t[9];
  if (!transposed) {
    for (int r = 0; r < nb; ++r) {
      double s = v[o + r];
      for (int q = 0; q < r; ++q) s -= L[r][q] * t[q];
      t[r] = s / L[r][r];
    }
  } else {
    for (int r = nb - 1; r >= 0; --r) {
      double s = v[o + r];
      for (int q = r + 1; q < nb; ++q) s -= L[q][r] * t[q];
      t[r] = s / L[r][r];
    }
  }
  for (int r = 0; r < nb; ++r) y[o + r] = t[r];
}

}  // namespace

// ===========================================================================
struct ba_gnn {
  int cd = 9, prec = 1, device = 0;
  std::string err;
  Layout L;
  hipStream_t stream = nullptr;  // own stream (training, batch evaluation)
  hipStream_t cur = nullptr;     // stream the launches go to
  float *params = nullptr, *grad = nullptr, *am = nullptr, *av = nullptr;
  uint16_t* pbf = nullptr;  // BF16 copy of the parameters
  int adam_t = 0;
  bool loaded = false;
  bool attached_training = false;  // the batch buffers hold a training batch, not the attached graph
  // batch buffers (capacity in nodes, edges, systems, S entries)
  int cap_n = 0, cap_m = 0, cap_g = 0;
  bool cap_train = false;  // the edge buffers of the backward pass exist
  int64_t cap_sn = 0, cap_se = 0;
  float *X = nullptr, *Zin = nullptr, *Hs = nullptr /*4 x n x H*/, *Ph = nullptr /*LAYERS x n x H*/,
        *Ze = nullptr /*LAYERS x m x H, training only*/, *Mm = nullptr, *Zs = nullptr, *heads = nullptr, *dheads = nullptr, *dH = nullptr,
        *dH2 = nullptr, *dZ = nullptr, *dE = nullptr, *ex = nullptr, *unit = nullptr;
  uint16_t *bfA = nullptr, *bfB = nullptr;  // BF16 operand scratch
  int32_t *type = nullptr, *graph = nullptr, *src = nullptr, *dst = nullptr, *rev = nullptr, *dst_off = nullptr;
  int2* runs = nullptr;  // edge runs of the message kernel (node, first edge)
  int n_runs = 0;
  std::vector<int32_t> h_off;  // host copies kept alive across the asynchronous uploads
  std::vector<int2> h_runs;
  double *SZ = nullptr, *DZ = nullptr, *Ag = nullptr, *Q1 = nullptr, *Q2 = nullptr, *gauge = nullptr;
  double *s_node = nullptr, *s_edge = nullptr;
  int64_t *s_node_off = nullptr, *s_edge_off = nullptr;
  double* scal = nullptr;  // loss, systems skipped
  // attached problem graph (inference)
  int gn = 0, gm = 0, type_end[3] = {0, 0, 0};
  double s0 = 1.0;
  float* gstat = nullptr;
  int2* etyped = nullptr;  // per edge of the attached graph: (log1p(shared records) bits, kind 1..4)
  std::vector<void*> allocs;
};

namespace {

template <typename P> P* dalloc(ba_gnn* g, size_t count) {
  void* p = nullptr;
  GCHK(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(P)));
  g->allocs.push_back(p);
  return (P*)p;
}
void dfree(ba_gnn* g, void* p) {
  if (!p) return;
  (void)hipFree(p);
  g->allocs.erase(std::remove(g->allocs.begin(), g->allocs.end(), p), g->allocs.end());
}

void reserve(ba_gnn* g, int n, int m, int G, int64_t sn, int64_t se, bool train) {
  if (n <= g->cap_n && m <= g->cap_m && G <= g->cap_g && sn <= g->cap_sn && se <= g->cap_se && (!train || g->cap_train))
    return;
  train = train || g->cap_train;
  n = std::max(n, g->cap_n); m = std::max(m, g->cap_m); G = std::max(G, g->cap_g);
  sn = std::max(sn, g->cap_sn); se = std::max(se, g->cap_se);
  float** fl[] = {&g->X, &g->Zin, &g->Hs, &g->Ph, &g->Ze, &g->Mm, &g->Zs, &g->heads, &g->dheads,
                  &g->dH, &g->dH2, &g->dZ, &g->dE, &g->ex, &g->unit};
  for (float** p : fl) { dfree(g, *p); *p = nullptr; }
  int32_t** il[] = {&g->type, &g->graph, &g->src, &g->dst, &g->rev, &g->dst_off};
  for (int32_t** p : il) { dfree(g, *p); *p = nullptr; }
  double** dl[] = {&g->SZ, &g->DZ, &g->Ag, &g->Q1, &g->Q2, &g->s_node, &g->s_edge, &g->gauge};
  for (double** p : dl) { dfree(g, *p); *p = nullptr; }
  dfree(g, g->bfA); dfree(g, g->bfB); dfree(g, g->s_node_off); dfree(g, g->s_edge_off); dfree(g, g->runs);
  const size_t nh = (size_t)n * H, mh = (size_t)m * H;
  g->X = dalloc<float>(g, (size_t)n * NIN);
  g->Zin = dalloc<float>(g, nh);
  g->Hs = dalloc<float>(g, (LAYERS + 1) * nh);
  g->Ph = dalloc<float>(g, (size_t)LAYERS * nh);
  g->Ze = dalloc<float>(g, train ? (size_t)LAYERS * mh : 1);
  g->Mm = dalloc<float>(g, (size_t)LAYERS * nh);
  g->Zs = dalloc<float>(g, (size_t)LAYERS * nh);
  g->heads = dalloc<float>(g, (size_t)n * HEADP);
  g->dheads = dalloc<float>(g, (size_t)n * HEADP);
  g->dH = dalloc<float>(g, nh);
  g->dH2 = dalloc<float>(g, nh);
  g->dZ = dalloc<float>(g, nh);
  g->dE = dalloc<float>(g, train ? mh : 1);
  g->ex = dalloc<float>(g, (size_t)m * EIN);
  g->unit = dalloc<float>(g, (size_t)n * 9);
  const size_t big = std::max({train ? mh : 1, (size_t)m * EIN, nh, (size_t)n * HEADP});
  g->bfA = dalloc<uint16_t>(g, big);
  g->bfB = dalloc<uint16_t>(g, big);
  g->type = dalloc<int32_t>(g, n); g->graph = dalloc<int32_t>(g, n);
  g->src = dalloc<int32_t>(g, m); g->dst = dalloc<int32_t>(g, m); g->rev = dalloc<int32_t>(g, m);
  g->dst_off = dalloc<int32_t>(g, n + 1);
  g->runs = dalloc<int2>(g, (size_t)m / EDGE_RUN + n + 1);
  g->SZ = dalloc<double>(g, (size_t)n * 9 * KT);
  g->DZ = dalloc<double>(g, (size_t)n * 9 * KT);
  g->Ag = dalloc<double>(g, (size_t)2 * G * KT * KT);  // A then G
  g->Q1 = dalloc<double>(g, (size_t)G * KT * KT);
  g->Q2 = dalloc<double>(g, (size_t)G * KT * KT);
  g->gauge = dalloc<double>(g, (size_t)n * 9 * KG);
  g->s_node = dalloc<double>(g, sn);
  g->s_edge = dalloc<double>(g, se);
  g->s_node_off = dalloc<int64_t>(g, n);
  g->s_edge_off = dalloc<int64_t>(g, m);
  g->cap_n = n; g->cap_m = m; g->cap_g = G; g->cap_sn = sn; g->cap_se = se; g->cap_train = train;
}

// C = A B  (A: M x K, B: K x N); operands FP32 in device memory with the given strides.
// In BF16 precision the operands are rounded to BF16 first (into bfA / bfB).
void gemm(ba_gnn* g, int M, int N, int K, const float* A, int64_t as0, int64_t as1, const float* B, int64_t bs0,
          int64_t bs1, float* C, int ldc, int mode, bool b_is_param = false, size_t b_param_off = 0) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
  int ksplit = 1;
  if (tiles < 256) ksplit = std::max(1, std::min(64, K / 256));
  // split-K accumulates with atomics into C (cleared first when C is overwritten)
  int eff_mode = mode;
  if (ksplit > 1) {
    if (mode == 0)
      hipLaunchKernelGGL(k_fill2d, dim3(nblk((int64_t)M * N, 256)), dim3(256), 0, g->cur, C, M, N, ldc);
    eff_mode = 2;
  }
  const int64_t threads = (int64_t)tiles * ksplit * 64;
  if (g->prec == 1) {
    // BF16 copies of the operands (parameters have a persistent copy)
    const int64_t a_elems = (int64_t)(M - 1) * as0 + (int64_t)(K - 1) * as1 + 1;
    hipLaunchKernelGGL(k_cast_bf16, dim3(nblk(a_elems, 256)), dim3(256), 0, g->cur, A, g->bfA, a_elems);
    const uint16_t* Bb;
    if (b_is_param) Bb = g->pbf + b_param_off;
    else {
      const int64_t b_elems = (int64_t)(K - 1) * bs0 + (int64_t)(N - 1) * bs1 + 1;
      hipLaunchKernelGGL(k_cast_bf16, dim3(nblk(b_elems, 256)), dim3(256), 0, g->cur, B, g->bfB, b_elems);
      Bb = g->bfB;
    }
    View Av{g->bfA, as0, as1}, Bv{Bb, bs0, bs1};
    hipLaunchKernelGGL(k_gemm<true>, dim3(nblk(threads, 256)), dim3(256), 0, g->cur, M, N, K, Av, Bv, C, ldc, ksplit, eff_mode);
  } else {
    View Av{A, as0, as1}, Bv{B, bs0, bs1};
    hipLaunchKernelGGL(k_gemm<false>, dim3(nblk(threads, 256)), dim3(256), 0, g->cur, M, N, K, Av, Bv, C, ldc, ksplit, eff_mode);
  }
}

void refresh_bf16_params(ba_gnn* g) {
  if (g->prec == 1)
    hipLaunchKernelGGL(k_cast_bf16, dim3(nblk(g->L.total, 256)), dim3(256), 0, g->cur, g->params, g->pbf,
                       (int64_t)g->L.total);
}

struct Dims {
  int n, m, type_end[3];
};

// forward over the batch currently in the device buffers
// forward over the batch (or attached graph) in the device buffers; keep_edges stores
// the edge pre-activations for the backward pass; typed: the attached graph's edges, with
// the (value, kind) words of k_edge_msg_typed
void forward(ba_gnn* g, const Dims& D, bool keep_edges, bool typed = false) {
  const int n = D.n, m = D.m;
  const Layout& L = g->L;
  const float* P = g->params;
  float* h0 = g->Hs;
  // input layer
  gemm(g, n, H, NIN, g->X, NIN, 1, P + L.W_in, H, 1, g->Zin, H, 0, true, L.W_in);
  hipLaunchKernelGGL(k_bias_act, dim3(nblk((int64_t)n * H, 256)), dim3(256), 0, g->cur, g->Zin, P + L.b_in,
                     (const float*)nullptr, (const float*)nullptr, h0, n, H);
  for (int l = 0; l < LAYERS; ++l) {
    float* hl = g->Hs + (size_t)l * n * H;
    float* hn = g->Hs + (size_t)(l + 1) * n * H;
    float* Ph = g->Ph + (size_t)l * n * H;
    float* Mm = g->Mm + (size_t)l * n * H;
    float* Zs = g->Zs + (size_t)l * n * H;
    // messages: the h-part of W_e applied per node, then one pass over the edges
    gemm(g, n, H, H, hl, H, 1, P + L.W_e[l], H, 1, Ph, H, 0, true, L.W_e[l]);
    GCHK(hipMemsetAsync(Mm, 0, (size_t)n * H * sizeof(float), g->cur));
    if (g->n_runs > 0 && typed)
      hipLaunchKernelGGL(k_edge_msg_typed, dim3(nblk((int64_t)g->n_runs * H, 256)), dim3(256), 0, g->cur, (const float*)Ph,
                         (const int2*)g->etyped, P + L.W_e[l] + (size_t)H * H, P + L.b_e[l], (const int32_t*)g->src,
                         (const int32_t*)g->dst_off, (const int2*)g->runs, g->n_runs, Mm);
    else if (g->n_runs > 0)
      hipLaunchKernelGGL(k_edge_msg, dim3(nblk((int64_t)g->n_runs * H, 256)), dim3(256), 0, g->cur, (const float*)Ph,
                         (const float*)g->ex, P + L.W_e[l] + (size_t)H * H, P + L.b_e[l], (const int32_t*)g->src,
                         (const int32_t*)g->dst_off, (const int2*)g->runs, g->n_runs,
                         keep_edges && m > 0 ? g->Ze + (size_t)l * m * H : (float*)nullptr, Mm);
    gemm(g, n, H, H, hl, H, 1, P + L.W_s[l], H, 1, Zs, H, 0, true, L.W_s[l]);
    hipLaunchKernelGGL(k_bias_act, dim3(nblk((int64_t)n * H, 256)), dim3(256), 0, g->cur, Zs, P + L.b_s[l],
                       (const float*)Mm, (const float*)hl, hn, n, H);
  }
  const float* hL = g->Hs + (size_t)LAYERS * n * H;
  GCHK(hipMemsetAsync(g->heads, 0, (size_t)n * HEADP * sizeof(float), g->cur));
  int b = 0;
  for (int t = 0; t < 3; ++t) {
    const int e = D.type_end[t];
    if (e > b) {
      gemm(g, e - b, L.T[t], H, hL + (size_t)b * H, H, 1, P + L.W_t[t], L.T[t], 1, g->heads + (size_t)b * HEADP, HEADP,
           0, true, L.W_t[t]);
      hipLaunchKernelGGL(k_bias_add, dim3(nblk((int64_t)(e - b) * L.T[t], 256)), dim3(256), 0, g->cur,
                         g->heads + (size_t)b * HEADP, P + L.b_t[t], e - b, L.T[t], HEADP);
    }
    b = e;
  }
}

void colsum(ba_gnn* g, const float* X, int rows, int cols, int ld, float* out) {
  if (rows <= 0) return;
  dim3 grid(std::min(256u, nblk(rows, 4)), (cols + 63) / 64);
  hipLaunchKernelGGL(k_colsum, grid, dim3(256), 0, g->cur, X, rows, cols, ld, out);
}

// backward from g->dheads into g->grad (zeroed by the caller)
void backward(ba_gnn* g, const Dims& D) {
  const int n = D.n, m = D.m;
  const Layout& L = g->L;
  const float* P = g->params;
  float* G = g->grad;
  const float* hL = g->Hs + (size_t)LAYERS * n * H;
  GCHK(hipMemsetAsync(g->dH, 0, (size_t)n * H * sizeof(float), g->cur));
  int b = 0;
  for (int t = 0; t < 3; ++t) {
    const int e = D.type_end[t];
    if (e > b) {
      const int rows = e - b, T = L.T[t];
      const float* dA = g->dheads + (size_t)b * HEADP;
      // dW_t += h^T dA ; db_t += colsum dA ; dh += dA W_t^T
      gemm(g, H, T, rows, hL + (size_t)b * H, 1, H, dA, HEADP, 1, G + L.W_t[t], T, 2);
      colsum(g, dA, rows, T, HEADP, G + L.b_t[t]);
      gemm(g, rows, H, T, dA, HEADP, 1, P + L.W_t[t], 1, T, g->dH + (size_t)b * H, H, 1);
    }
    b = e;
  }
  float* dh = g->dH;   // gradient w.r.t. h_{l+1}
  float* dh2 = g->dH2; // gradient w.r.t. h_l
  for (int l = LAYERS - 1; l >= 0; --l) {
    const float* hl = g->Hs + (size_t)l * n * H;
    const float* Ze = g->Ze + (size_t)l * m * H;
    const float* Zs = g->Zs + (size_t)l * n * H;
    float* dZ = g->dZ;
    // node update: h_{l+1} = gelu(Zs) + h_l, Zs = h_l W_s + b_s + m
    hipLaunchKernelGGL(k_act_bwd, dim3(nblk((int64_t)n * H, 256)), dim3(256), 0, g->cur, dh, Zs, dZ, (int64_t)n * H);
    gemm(g, H, H, n, hl, 1, H, dZ, H, 1, G + L.W_s[l], H, 2);
    colsum(g, dZ, n, H, H, G + L.b_s[l]);
    GCHK(hipMemcpyAsync(dh2, dh, (size_t)n * H * sizeof(float), hipMemcpyDeviceToDevice, g->cur));
    gemm(g, n, H, H, dZ, H, 1, P + L.W_s[l], 1, H, dh2, H, 1, true, L.W_s[l]);
    if (m > 0) {
      // messages: dZe = dm[dst] / deg * gelu'(Ze); db_e, dW_x = e^T dZe, dP[src] += dZe,
      // dW_h = h^T dP, dh += dP W_h^T
      float* dZe = g->dE;
      hipLaunchKernelGGL(k_edge_msg_bwd, dim3(nblk((int64_t)m * H, 256)), dim3(256), 0, g->cur, (const float*)dZ, Ze,
                         (const int32_t*)g->dst, (const int32_t*)g->dst_off, dZe, m);
      colsum(g, dZe, m, H, H, G + L.b_e[l]);
      gemm(g, EIN, H, m, g->ex, 1, EIN, dZe, H, 1, G + L.W_e[l] + (size_t)H * H, H, 2);
      float* dP = g->dZ;  // dZs is consumed
      hipLaunchKernelGGL(k_scatter_src, dim3(nblk((int64_t)n * H, 256)), dim3(256), 0, g->cur, (const float*)dZe,
                         (const int32_t*)g->rev, (const int32_t*)g->dst_off, dP, n);
      gemm(g, H, H, n, hl, 1, H, dP, H, 1, G + L.W_e[l], H, 2);
      gemm(g, n, H, H, dP, H, 1, P + L.W_e[l], 1, H, dh2, H, 1, true, L.W_e[l]);
    }
    std::swap(dh, dh2);
  }
  // input layer: h0 = gelu(Zin)
  hipLaunchKernelGGL(k_act_bwd, dim3(nblk((int64_t)n * H, 256)), dim3(256), 0, g->cur, dh, g->Zin, g->dZ, (int64_t)n * H);
  gemm(g, NIN, H, n, g->X, 1, NIN, g->dZ, H, 1, G + L.W_in, H, 2);
  colsum(g, g->dZ, n, H, H, G + L.b_in);
}

int bsize(const ba_gnn* g, int type) { return type == 0 ? g->cd : type == 1 ? 3 : 2; }

bool check_batch(ba_gnn* g, const ba_gnn_batch* b, bool need_s) {
  if (!b || b->n_nodes <= 0 || b->n_edges < 0 || b->n_graphs <= 0 || !b->node_x || !b->node_type ||
      !b->node_graph || !b->node_unit ||
      (b->n_edges > 0 && (!b->edge_src || !b->edge_dst || !b->edge_rev || !b->edge_x))) {
    g->err = "batch sizes or arrays missing";
    return false;
  }
  for (int i = 0; i < b->n_nodes; ++i) {
    if (b->node_type[i] < 0 || b->node_type[i] > 2 || (i && b->node_type[i] < b->node_type[i - 1])) {
      g->err = "node types must be 0..2 and sorted";
      return false;
    }
    if (b->node_graph[i] < 0 || b->node_graph[i] >= b->n_graphs) {
      g->err = "node system id out of range";
      return false;
    }
  }
  for (int e = 0; e < b->n_edges; ++e) {
    if (b->edge_src[e] < 0 || b->edge_src[e] >= b->n_nodes || b->edge_dst[e] < 0 || b->edge_dst[e] >= b->n_nodes ||
        b->edge_rev[e] < 0 || b->edge_rev[e] >= b->n_edges || (e && b->edge_dst[e] < b->edge_dst[e - 1]) ||
        b->edge_src[e] == b->edge_dst[e]) {
      g->err = "edges out of range, self-loops, or not sorted by destination";
      return false;
    }
  }
  for (int e = 0; e < b->n_edges; ++e) {
    const int r = b->edge_rev[e];
    if (b->edge_src[r] != b->edge_dst[e] || b->edge_dst[r] != b->edge_src[e] ||
        b->node_graph[b->edge_src[e]] != b->node_graph[b->edge_dst[e]]) {
      g->err = "edge_rev does not give each edge's reverse, or an edge joins two systems";
      return false;
    }
  }
  if (need_s) {
    if (!b->s_node || !b->s_node_off || (b->n_edges > 0 && (!b->s_edge || !b->s_edge_off)) || b->s_node_len <= 0 ||
        b->s_edge_len < 0 || !b->node_gauge) {
      g->err = "the loss needs the S blocks of every node and edge and the gauge blocks";
      return false;
    }
    for (int i = 0; i < b->n_nodes; ++i) {
      const int ni = bsize(g, b->node_type[i]);
      if (b->s_node_off[i] < 0 || b->s_node_off[i] + (int64_t)ni * ni > b->s_node_len) {
        g->err = "S block of a node out of range";
        return false;
      }
    }
    for (int e = 0; e < b->n_edges; ++e) {
      const int64_t sz = (int64_t)bsize(g, b->node_type[b->edge_dst[e]]) * bsize(g, b->node_type[b->edge_src[e]]);
      if (b->s_edge_off[e] < 0 || b->s_edge_off[e] + sz > b->s_edge_len) {
        g->err = "S block of an edge out of range";
        return false;
      }
    }
  }
  return true;
}

// runs of <= EDGE_RUN in-edges per node from the CSR offsets, uploaded with the offsets
void upload_runs(ba_gnn* g, const int32_t* off, int n, hipStream_t s) {
  g->h_off.assign(off, off + n + 1);
  g->h_runs.clear();
  for (int i = 0; i < n; ++i)
    for (int e = off[i]; e < off[i + 1]; e += EDGE_RUN) g->h_runs.push_back(make_int2(i, e));
  g->n_runs = (int)g->h_runs.size();
  GCHK(hipMemcpyAsync(g->dst_off, g->h_off.data(), g->h_off.size() * 4, hipMemcpyHostToDevice, s));
  if (g->n_runs) GCHK(hipMemcpyAsync(g->runs, g->h_runs.data(), g->h_runs.size() * sizeof(int2), hipMemcpyHostToDevice, s));
}

Dims upload_batch(ba_gnn* g, const ba_gnn_batch* b, bool with_s) {
  reserve(g, b->n_nodes, b->n_edges, b->n_graphs, with_s ? b->s_node_len : 1, with_s ? std::max<int64_t>(b->s_edge_len, 1) : 1,
          with_s);
  g->attached_training = true;
  g->cur = g->stream;
  Dims D;
  D.n = b->n_nodes;
  D.m = b->n_edges;
  std::vector<int32_t> off(D.n + 1, 0);
  for (int e = 0; e < D.m; ++e) off[b->edge_dst[e] + 1]++;
  for (int i = 0; i < D.n; ++i) off[i + 1] += off[i];
  int te[3] = {0, 0, 0};
  for (int i = 0; i < D.n; ++i) te[b->node_type[i]] = i + 1;
  D.type_end[0] = te[0];
  D.type_end[1] = std::max(te[1], D.type_end[0]);
  D.type_end[2] = std::max(te[2], D.type_end[1]);
  hipStream_t s = g->cur;
  GCHK(hipMemcpyAsync(g->X, b->node_x, (size_t)D.n * NIN * 4, hipMemcpyHostToDevice, s));
  GCHK(hipMemcpyAsync(g->type, b->node_type, (size_t)D.n * 4, hipMemcpyHostToDevice, s));
  GCHK(hipMemcpyAsync(g->graph, b->node_graph, (size_t)D.n * 4, hipMemcpyHostToDevice, s));
  GCHK(hipMemcpyAsync(g->unit, b->node_unit, (size_t)D.n * 9 * 4, hipMemcpyHostToDevice, s));
  if (D.m) {
    GCHK(hipMemcpyAsync(g->src, b->edge_src, (size_t)D.m * 4, hipMemcpyHostToDevice, s));
    GCHK(hipMemcpyAsync(g->dst, b->edge_dst, (size_t)D.m * 4, hipMemcpyHostToDevice, s));
    GCHK(hipMemcpyAsync(g->rev, b->edge_rev, (size_t)D.m * 4, hipMemcpyHostToDevice, s));
    GCHK(hipMemcpyAsync(g->ex, b->edge_x, (size_t)D.m * EIN * 4, hipMemcpyHostToDevice, s));
  }
  upload_runs(g, off.data(), D.n, s);
  if (with_s) {
    GCHK(hipMemcpyAsync(g->s_node, b->s_node, (size_t)b->s_node_len * 8, hipMemcpyHostToDevice, s));
    GCHK(hipMemcpyAsync(g->s_node_off, b->s_node_off, (size_t)D.n * 8, hipMemcpyHostToDevice, s));
    GCHK(hipMemcpyAsync(g->gauge, b->node_gauge, (size_t)D.n * 9 * KG * 8, hipMemcpyHostToDevice, s));
    if (D.m) {
      GCHK(hipMemcpyAsync(g->s_edge, b->s_edge, (size_t)b->s_edge_len * 8, hipMemcpyHostToDevice, s));
      GCHK(hipMemcpyAsync(g->s_edge_off, b->s_edge_off, (size_t)D.m * 8, hipMemcpyHostToDevice, s));
    }
  }
  return D;
}

// coarse loss of the heads in g->heads and its gradient into g->dheads
void coarse_loss(ba_gnn* g, const Dims& D, int n_graphs) {
  hipStream_t s = g->cur;
  GCHK(hipMemsetAsync(g->Ag, 0, (size_t)2 * n_graphs * KT * KT * 8, s));
  GCHK(hipMemsetAsync(g->scal, 0, 2 * 8, s));
  const int64_t np = (int64_t)D.n * 9 * KT;
  hipLaunchKernelGGL(k_coarse_products, dim3(nblk(np, 256)), dim3(256), 0, s, (const float*)g->heads,
                     (const float*)g->unit, (const double*)g->gauge, (const int32_t*)g->type, (const int32_t*)g->src,
                     (const int32_t*)g->dst_off, (const double*)g->s_node, (const int64_t*)g->s_node_off,
                     (const double*)g->s_edge, (const int64_t*)g->s_edge_off, D.n, g->cd, g->SZ, g->DZ);
  hipLaunchKernelGGL(k_coarse_gram, dim3(nblk((int64_t)D.n * KT * KT, 256)), dim3(256), 0, s, (const float*)g->heads,
                     (const float*)g->unit, (const double*)g->gauge, (const int32_t*)g->type, (const int32_t*)g->graph,
                     (const double*)g->SZ, (const double*)g->DZ, D.n, g->cd, g->Ag,
                     g->Ag + (size_t)n_graphs * KT * KT);
  hipLaunchKernelGGL(k_coarse_loss, dim3(nblk(n_graphs, 64)), dim3(64), 0, s, (const double*)g->Ag,
                     (const double*)(g->Ag + (size_t)n_graphs * KT * KT), n_graphs, g->Q1, g->Q2, g->scal, g->scal + 1);
  hipLaunchKernelGGL(k_coarse_dheads, dim3(nblk((int64_t)D.n * HEADP, 256)), dim3(256), 0, s, (const double*)g->SZ,
                     (const double*)g->DZ, (const double*)g->Q1, (const double*)g->Q2, (const float*)g->unit,
                     (const int32_t*)g->type, (const int32_t*)g->graph, D.n, g->cd, n_graphs, g->dheads);
}

}  // namespace

// ===========================================================================
namespace ba_gnn_impl {

size_t param_count(int cd) { return make_layout(cd).total; }

ba_gnn* create(int cd, int precision, int device, std::string& err) {
  ba_gnn* g = new ba_gnn();
  try {
    g->cd = cd;
    g->prec = precision;
    g->device = device;
    g->L = make_layout(cd);
    GCHK(hipSetDevice(device));
    GCHK(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
    g->cur = g->stream;
    g->params = dalloc<float>(g, g->L.total);
    g->grad = dalloc<float>(g, g->L.total);
    g->am = dalloc<float>(g, g->L.total);
    g->av = dalloc<float>(g, g->L.total);
    g->pbf = dalloc<uint16_t>(g, g->L.total);
    g->scal = dalloc<double>(g, 2);
    GCHK(hipMemsetAsync(g->params, 0, g->L.total * 4, g->cur));
    GCHK(hipMemsetAsync(g->am, 0, g->L.total * 4, g->cur));
    GCHK(hipMemsetAsync(g->av, 0, g->L.total * 4, g->cur));
    GCHK(hipStreamSynchronize(g->cur));
  } catch (const std::exception& e) {
    err = e.what();
    destroy(g);
    return nullptr;
  }
  return g;
}

void destroy(ba_gnn* g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  for (void* p : g->allocs) (void)hipFree(p);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
}

bool load(ba_gnn* g, const void* blob, size_t bytes, std::string& err) {
  if (bytes != g->L.total * sizeof(float)) {
    err = "weight blob has " + std::to_string(bytes) + " bytes, expected " + std::to_string(g->L.total * sizeof(float));
    return false;
  }
  const float* f = (const float*)blob;
  for (size_t i = 0; i < g->L.total; ++i)
    if (!std::isfinite(f[i])) { err = "non-finite weight"; return false; }
  GCHK(hipSetDevice(g->device));
  g->cur = g->stream;
  GCHK(hipMemcpyAsync(g->params, blob, bytes, hipMemcpyHostToDevice, g->stream));
  refresh_bf16_params(g);
  GCHK(hipStreamSynchronize(g->stream));
  g->loaded = true;
  g->adam_t = 0;
  return true;
}

bool ready(const ba_gnn* g) { return g && g->loaded && g->gn > 0 && !g->attached_training; }

void build_graph(Graph& G, int nc, int ng, int nv, int cd, const std::vector<int64_t>& fb_off,
                 const std::vector<int32_t>& fb, const std::vector<int64_t>& block_records, double scale) {
  const int n = nc + ng + nv;
  G = Graph();
  if (n == 0 || n > MAX_GRAPH_NODES) return;
  // shared-feature counts of every ordered block pair
  std::vector<int32_t> cnt((size_t)n * n, 0);
  const size_t nf = fb_off.empty() ? 0 : fb_off.size() - 1;
  for (size_t f = 0; f < nf; ++f)
    for (int64_t a = fb_off[f]; a < fb_off[f + 1]; ++a)
      for (int64_t b = fb_off[f]; b < fb_off[f + 1]; ++b)
        if (a != b) cnt[(size_t)fb[a] * n + fb[b]]++;
  G.n_nodes = n;
  G.node_type.resize(n);
  G.node_off.resize(n);
  G.node_size.resize(n);
  for (int i = 0; i < n; ++i) {
    G.node_type[i] = i < nc ? 0 : i < nc + ng ? 1 : 2;
    G.node_size[i] = i < nc ? cd : i < nc + ng ? 3 : 2;
    G.node_off[i] = i < nc ? cd * i : i < nc + ng ? cd * nc + 3 * (i - nc) : cd * nc + 3 * ng + 2 * (i - nc - ng);
  }
  // edges sorted by destination, then source
  G.dst_off.assign(n + 1, 0);
  std::vector<int32_t> deg(n, 0);
  for (int d = 0; d < n; ++d) {
    for (int s = 0; s < n; ++s) {
      const int32_t c = cnt[(size_t)s * n + d];
      if (!c) continue;
      G.edge_src.push_back(s);
      G.edge_dst.push_back(d);
      const int ts = G.node_type[s], td = G.node_type[d];
      float ef[EDGE_IN] = {0};
      ef[0] = std::log1p((float)c);
      if (ts == 0 && td == 0) ef[1] = 1;
      else if (ts + td == 1) ef[2] = 1;       // camera - plane
      else if (ts == 0 || td == 0) ef[3] = 1; // camera - VP
      else ef[4] = 1;                          // group - group
      G.edge_x.insert(G.edge_x.end(), ef, ef + EDGE_IN);
      int kind = 1;
      while (kind < 4 && ef[kind] == 0.0f) ++kind;
      int32_t bits;
      std::memcpy(&bits, &ef[0], sizeof(bits));
      G.edge_typed.push_back(make_int2(bits, kind));
      deg[d]++;
    }
    G.dst_off[d + 1] = (int32_t)G.edge_src.size();
  }
  G.n_edges = (int)G.edge_src.size();
  // reverse of (s -> d) is (d -> s): in the in-list of s, sorted by source
  G.edge_rev.assign(G.n_edges, 0);
  for (int e = 0; e < G.n_edges; ++e) {
    const int s = G.edge_src[e], d = G.edge_dst[e];
    const auto b = G.edge_src.begin() + G.dst_off[s], en = G.edge_src.begin() + G.dst_off[s + 1];
    G.edge_rev[e] = (int32_t)(std::lower_bound(b, en, d) - G.edge_src.begin());
  }
  G.node_static.assign((size_t)n * NODE_IN, 0.0f);
  for (int i = 0; i < n; ++i) {
    float* x = &G.node_static[(size_t)i * NODE_IN];
    x[46] = std::log1p((float)block_records[i]);
    x[47] = std::log1p((float)deg[i]);
    x[48 + G.node_type[i]] = 1.0f;
  }
  G.scale = scale;
  G.valid = true;
}

void attach(ba_gnn* g, const Graph& G) {
  if (!G.valid) return;
  GCHK(hipSetDevice(g->device));
  reserve(g, G.n_nodes, G.n_edges, 1, 1, 1, false);
  g->gn = G.n_nodes;
  g->gm = G.n_edges;
  g->s0 = G.scale;
  for (int t = 0; t < 3; ++t) g->type_end[t] = 0;
  for (int i = 0; i < G.n_nodes; ++i) g->type_end[G.node_type[i]] = i + 1;
  for (int t = 1; t < 3; ++t) g->type_end[t] = std::max(g->type_end[t], g->type_end[t - 1]);
  if (g->gstat) dfree(g, g->gstat);
  g->gstat = dalloc<float>(g, (size_t)G.n_nodes * NODE_IN);
  hipStream_t s = g->stream;
  GCHK(hipMemcpyAsync(g->gstat, G.node_static.data(), G.node_static.size() * 4, hipMemcpyHostToDevice, s));
  GCHK(hipMemcpyAsync(g->type, G.node_type.data(), G.n_nodes * 4, hipMemcpyHostToDevice, s));
  if (G.n_edges) {
    GCHK(hipMemcpyAsync(g->src, G.edge_src.data(), G.n_edges * 4, hipMemcpyHostToDevice, s));
    GCHK(hipMemcpyAsync(g->dst, G.edge_dst.data(), G.n_edges * 4, hipMemcpyHostToDevice, s));
    GCHK(hipMemcpyAsync(g->rev, G.edge_rev.data(), G.n_edges * 4, hipMemcpyHostToDevice, s));
    GCHK(hipMemcpyAsync(g->ex, G.edge_x.data(), G.edge_x.size() * 4, hipMemcpyHostToDevice, s));
  }
  if (g->etyped) dfree(g, g->etyped);
  g->etyped = dalloc<int2>(g, (size_t)G.n_edges);
  if (G.n_edges) GCHK(hipMemcpyAsync(g->etyped, G.edge_typed.data(), G.edge_typed.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  upload_runs(g, G.dst_off.data(), G.n_nodes, s);
  GCHK(hipStreamSynchronize(s));
  g->attached_training = false;
}

void launch_node_features(const ba::Dev& d, const float* stat, const int32_t* type, int n, double lambda, double s0,
                          float* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_node_features, dim3(nblk(n, 128)), dim3(128), 0, s, d, stat, type, n, lambda, s0, out);
}

void launch_block_tri(const ba::Dev& d, const double* v, double* y, bool transposed, hipStream_t s) {
  const int nb = d.nc + d.ng + d.nv;
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_block_tri, dim3(nblk(nb, 64)), dim3(64), 0, s, d, v, y, transposed ? 1 : 0);
}

void apply(ba_gnn* g, const ba::Dev& d, double lambda, hipStream_t s) {
  if (!ready(g)) throw std::runtime_error("no weights or no attached graph");
  g->cur = s;  // ordered after the solver's assembly on its stream
  launch_node_features(d, g->gstat, g->type, g->gn, lambda, g->s0, g->X, s);
  Dims D{g->gn, g->gm, {g->type_end[0], g->type_end[1], g->type_end[2]}};
  forward(g, D, false, g->etyped != nullptr);
  hipLaunchKernelGGL(k_coarse_basis, dim3(nblk((int64_t)g->gn * HEADP, 256)), dim3(256), 0, s, d,
                     (const float*)g->heads, (const int32_t*)g->type, g->gn, g->s0);
  g->cur = g->stream;
}

}  // namespace ba_gnn_impl

// ===========================================================================
// C ABI of the network and its trainer
extern "C" {

size_t ba_gnn_param_count(int32_t camera_dof) { return make_layout(camera_dof).total; }

ba_status ba_gnn_create(int32_t camera_dof, int32_t precision, int32_t device, ba_gnn** out) {
  if (!out) return BA_E_INVALID;
  *out = nullptr;
  if ((camera_dof != 6 && camera_dof != 9) || (precision != 0 && precision != 1)) return BA_E_INVALID;
  std::string err;
  ba_gnn* g = ba_gnn_impl::create(camera_dof, precision, device, err);
  if (!g) return BA_E_DEVICE;
  *out = g;
  return BA_OK;
}

ba_status ba_gnn_set_params(ba_gnn* g, const float* p, size_t count) {
  if (!g || !p) return BA_E_INVALID;
  std::string err;
  try {
    if (!ba_gnn_impl::load(g, p, count * sizeof(float), err)) { g->err = err; return BA_E_INVALID; }
  } catch (const std::exception& e) { g->err = e.what(); return BA_E_DEVICE; }
  return BA_OK;
}

ba_status ba_gnn_get_params(const ba_gnn* gc, float* p, size_t count) {
  ba_gnn* g = const_cast<ba_gnn*>(gc);
  if (!g || !p || count != g->L.total) return BA_E_INVALID;
  if (hipSetDevice(g->device) != hipSuccess) return BA_E_DEVICE;
  if (hipMemcpy(p, g->params, count * 4, hipMemcpyDeviceToHost) != hipSuccess) return BA_E_DEVICE;
  return BA_OK;
}

ba_status ba_gnn_forward(ba_gnn* g, const ba_gnn_batch* b, float* heads, double* loss) {
  if (!g) return BA_E_INVALID;
  const bool with_loss = loss != nullptr;
  if (!check_batch(g, b, with_loss)) return BA_E_INVALID;
  try {
    GCHK(hipSetDevice(g->device));
    Dims D = upload_batch(g, b, with_loss);
    forward(g, D, false);
    if (with_loss) {
      coarse_loss(g, D, b->n_graphs);
      GCHK(hipMemcpyAsync(loss, g->scal, 8, hipMemcpyDeviceToHost, g->cur));
    }
    if (heads) GCHK(hipMemcpyAsync(heads, g->heads, (size_t)D.n * HEADP * 4, hipMemcpyDeviceToHost, g->cur));
    GCHK(hipGetLastError());
    GCHK(hipStreamSynchronize(g->cur));
  } catch (const std::exception& e) {
    g->err = e.what();
    return BA_E_DEVICE;
  }
  return BA_OK;
}

ba_status ba_gnn_train_step(ba_gnn* g, const ba_gnn_batch* b, double lr, double* loss, float* grad) {
  if (!g) return BA_E_INVALID;
  if (!check_batch(g, b, true)) return BA_E_INVALID;
  try {
    GCHK(hipSetDevice(g->device));
    Dims D = upload_batch(g, b, true);
    forward(g, D, true);
    coarse_loss(g, D, b->n_graphs);
    GCHK(hipMemsetAsync(g->grad, 0, g->L.total * 4, g->cur));
    backward(g, D);
    if (lr > 0) {
      g->adam_t++;
      const float b1 = 0.9f, b2 = 0.999f;
      hipLaunchKernelGGL(k_adam, dim3(nblk(g->L.total, 256)), dim3(256), 0, g->cur, g->params, (const float*)g->grad,
                         g->am, g->av, (int64_t)g->L.total, (float)lr, b1, b2, 1e-8f,
                         1.0f - std::pow(b1, (float)g->adam_t), 1.0f - std::pow(b2, (float)g->adam_t));
      refresh_bf16_params(g);
    }
    if (loss) GCHK(hipMemcpyAsync(loss, g->scal, 8, hipMemcpyDeviceToHost, g->cur));
    if (grad) GCHK(hipMemcpyAsync(grad, g->grad, g->L.total * 4, hipMemcpyDeviceToHost, g->cur));
    GCHK(hipGetLastError());
    GCHK(hipStreamSynchronize(g->cur));
  } catch (const std::exception& e) {
    g->err = e.what();
    return BA_E_DEVICE;
  }
  return BA_OK;
}

const char* ba_gnn_last_error(const ba_gnn* g) { return g ? g->err.c_str() : "null network"; }

void ba_gnn_destroy(ba_gnn* g) { ba_gnn_impl::destroy(g); }

}  // extern "C"
