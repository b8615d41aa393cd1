// Host side of libba: the C ABI, input validation, the one-time expansion of
// associations into residual records (the analogue of the symbolic phase of
// the paper's Sec. 4.1), device buffer management and the Levenberg-Marquardt
// driver around the kernels of ba_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <numeric>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ba.h"
#include "ba_internal.h"
#include "ba_gnn.h"

using namespace ba;

// Device scratch of ba_export_schur_dense_noalloc: one panel of columns of the
// reduced matrix is formed here and copied out before the next.  Each GPU the
// library runs on holds its own copy until the process ends; in host code the
// name is only a stand-in, the device address comes from hipGetSymbolAddress.
constexpr int64_t NOALLOC_SCRATCH_DOUBLES = int64_t(1) << 19;  // 4 MiB
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {

struct BaError : std::runtime_error {
  ba_status code;
  BaError(ba_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(call)                                                                         \
  do {                                                                                       \
    hipError_t _e = (call);                                                                  \
    if (_e != hipSuccess)                                                                    \
      throw BaError(BA_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(_e));        \
  } while (0)

constexpr int PCG_CHECK_EVERY = 8;

// device address of `scratch` per device, taken once with that device current
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;

double* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) return it->second;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw BaError(BA_E_DEVICE, "no device address for the no-allocation scratch");
  g_scratch_ptr[device] = static_cast<double*>(p);
  return static_cast<double*>(p);
}

// ---------------------------------------------------------------------------
// parameter conversions (FP64, host)
void quat_to_R(const double* q0, double* R) {
  double n = std::sqrt(q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2] + q0[3] * q0[3]);
  double w = q0[0] / n, x = q0[1] / n, y = q0[2] / n, z = q0[3] / n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

void R_to_quat(const double* m, double* q) {
  double tr = m[0] + m[4] + m[8];
  if (tr > 0) {
    double s = std::sqrt(tr + 1.0) * 2;
    q[0] = 0.25 * s; q[1] = (m[7] - m[5]) / s; q[2] = (m[2] - m[6]) / s; q[3] = (m[3] - m[1]) / s;
  } else if (m[0] > m[4] && m[0] > m[8]) {
    double s = std::sqrt(1.0 + m[0] - m[4] - m[8]) * 2;
    q[0] = (m[7] - m[5]) / s; q[1] = 0.25 * s; q[2] = (m[1] + m[3]) / s; q[3] = (m[2] + m[6]) / s;
  } else if (m[4] > m[8]) {
    double s = std::sqrt(1.0 + m[4] - m[0] - m[8]) * 2;
    q[0] = (m[2] - m[6]) / s; q[1] = (m[1] + m[3]) / s; q[2] = 0.25 * s; q[3] = (m[5] + m[7]) / s;
  } else {
    double s = std::sqrt(1.0 + m[8] - m[0] - m[4]) * 2;
    q[0] = (m[3] - m[1]) / s; q[1] = (m[2] + m[6]) / s; q[2] = (m[5] + m[7]) / s; q[3] = 0.25 * s;
  }
  if (q[0] < 0) for (int i = 0; i < 4; ++i) q[i] = -q[i];
  double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int i = 0; i < 4; ++i) q[i] /= n;
}

void cross(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
double norm3(const double* a) { return std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

// unit vector orthogonal to u: normalise(e_k - (e_k . u) u), k = argmin |u_k|
void ortho_unit(const double* u, double* o) {
  int k = 0;
  if (std::fabs(u[1]) < std::fabs(u[k])) k = 1;
  if (std::fabs(u[2]) < std::fabs(u[k])) k = 2;
  for (int i = 0; i < 3; ++i) o[i] = (i == k ? 1.0 : 0.0) - u[k] * u[i];
  double n = norm3(o);
  for (int i = 0; i < 3; ++i) o[i] /= n;
}

// orthonormal line representation from two points: slot u1 u2 u3 w1 w2 pad
bool line_from_points(const double* P, const double* Q, double* slot) {
  double d[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]}, m[3];
  cross(P, d, m);
  double nd = norm3(d), nm = norm3(m);
  if (!(nd > 0) || !std::isfinite(nd) || !std::isfinite(nm)) return false;
  double u1[3] = {d[0] / nd, d[1] / nd, d[2] / nd}, u2[3], u3[3];
  if (nm < 1e-12 * nd) {
    ortho_unit(u1, u2);
    nm = 0;
  } else {
    for (int i = 0; i < 3; ++i) u2[i] = m[i] / nm;
  }
  cross(u1, u2, u3);
  double s = std::sqrt(nd * nd + nm * nm);
  for (int i = 0; i < 3; ++i) { slot[i] = u1[i]; slot[3 + i] = u2[i]; slot[6 + i] = u3[i]; }
  slot[9] = nd / s; slot[10] = nm / s; slot[11] = 0;
  return true;
}

void sphere_basis(const double* n, double* b1, double* b2) {
  ortho_unit(n, b1);
  cross(n, b1, b2);
}

// ---------------------------------------------------------------------------
struct DevAlloc {
  std::vector<void*> ptrs;
  template <typename P> P* get(size_t count, size_t elem = sizeof(P)) {
    if (count == 0) count = 1;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, count * elem);
    if (e != hipSuccess) throw BaError(BA_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    ptrs.push_back(p);
    return (P*)p;
  }
  void free_all() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

struct Obs {
  std::vector<int32_t> a, b;
  std::vector<double> meas;
  ba_loss loss;
  bool loss_set = false;
};

}  // namespace

struct ba_handle {
  // problem
  int nc = 0, np = 0, nl = 0, ng = 0, nv = 0, ns = 0, CD = 9;
  double cx = 0, cy = 0;
  int precision = BA_PREC_MIXED, precond = BA_PC_BLOCK_JACOBI;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  // host FP64 parameters in the device layouts (original feature order)
  std::vector<double> cam, pt, ln, pl, vp, sh;  // sh: SH_STRIDE per shape (ba_shape.h)
  Obs obs[13];  // ba_kind 0..5 observations and associations, 6..9 inter-group relations,
                //  10 3D point-to-plane associations, 11 / 12 shape associations
  // inter-group relations: caller's (group a, group b) and kind 0..3 per record
  std::vector<int32_t> rel_ga, rel_gb, rel_kind;
  // state
  bool finalized = false, need_lin = true, have_cost = false, first_step = true;
  double lambda = 1e-4, nu = 2.0, E = 0, Epix = 0, last_lambda = 0;
  // internal permutations: internal feature id -> caller id and inverse
  std::vector<int32_t> pt_perm, pt_inv, ln_perm, ln_inv;
  // record keys per family in caller indices (camera, feature, other)
  std::vector<int64_t> keys[NFAM];
  Dev d;
  DevAlloc alloc;
  double* hscal = nullptr;  // pinned host mirror of d.scal
  // learned preconditioner: network (weights loaded by the caller) and the
  // block graph of the reduced system, built at the symbolic phase
  ba_gnn* gnn = nullptr;
  ba_gnn_impl::Graph graph;
  float* g_stat = nullptr;     // device copies of the structural node inputs and types
  int32_t* g_type = nullptr;
  float* g_x = nullptr;        // node input features of the last linearisation
  hipEvent_t ev[BA_PHASE_COUNT + 1] = {};
  bool events = false;
  std::vector<hipEvent_t> mv_ev;  // pool for per-product timing
  // dense Schur solver: host tables of the (feature, block) entries and block pairs,
  // built at the symbolic phase for reduced systems of at most DENSE_MAX_NA rows and
  // uploaded, with the matrix storage, on first use
  struct DenseHost {
    bool built = false, uploaded = false;
    std::string why = "the dense solver's tables have not been built";
    std::vector<int2> fent, pair_ab, pair_ent, pair_u, chunk;
    std::vector<int32_t> pair_off, pair_uoff, pair_choff;
  } dense;
};

namespace {

ba_loss default_loss(int kind) {
  switch (kind) {
    case BA_ASSOC_PLANE_POINT: case BA_ASSOC_PLANE_LINE: case BA_ASSOC_SHAPE_POINT: case BA_ASSOC_SHAPE_LINE:
      return {BA_LOSS_CAUCHY, 1.0, 0.5};
    case BA_ASSOC_VP_LINE: return {BA_LOSS_CAUCHY, 0.2, 5.0e3};
    case BA_ASSOC_JUNCTION: return {BA_LOSS_CAUCHY, 1.0, 0.1};
    case BA_REL_VP_ORTHO: case BA_REL_VP_PARALLEL: case BA_REL_PLANE_ORTHO: case BA_REL_PLANE_PARALLEL:
      return {BA_LOSS_CAUCHY, 0.2, 5.0e3};
    case BA_ASSOC_PLANE_POINT_3D: return {BA_LOSS_TRIVIAL, 1.0, 100.0};
    default: return {BA_LOSS_TRIVIAL, 1.0, 1.0};
  }
}

template <typename V> void upload(ba_handle* h, V* dst, const std::vector<V>& src) {
  if (!src.empty()) HIPCHK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice, h->stream));
}

void sync(ba_handle* h) { HIPCHK(hipStreamSynchronize(h->stream)); }

void set_device(ba_handle* h) { HIPCHK(hipSetDevice(h->device)); }

void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw BaError(BA_E_DEVICE, std::string(what) + ": kernel launch failed: " + hipGetErrorString(e));
}


// ---------------------------------------------------------------------------
// expansion of associations into records (visibility rules of Sec. 3.3-3.4)
struct Rec {
  int32_t feat;   // internal feature id
  int32_t cam;    // camera or -1
  int32_t other;  // group, or partner feature (caller id), or -1
  int32_t grp;    // group index stored on the device, or -1
  double meas[4];
  int64_t key[3];
};

struct CSR {
  std::vector<int64_t> off;
  std::vector<int32_t> cam, idx;  // per feature: cameras ascending, observation index
  bool has(int f, int c) const {
    auto b = cam.begin() + off[f], e = cam.begin() + off[f + 1];
    return std::binary_search(b, e, c);
  }
};

CSR build_csr(const Obs& o, int nfeat, const char* what) {
  CSR s;
  const size_t n = o.a.size();
  s.off.assign(nfeat + 1, 0);
  for (size_t i = 0; i < n; ++i) s.off[o.b[i] + 1]++;
  for (int f = 0; f < nfeat; ++f) s.off[f + 1] += s.off[f];
  std::vector<int64_t> pos(s.off.begin(), s.off.end() - 1);
  s.cam.resize(n);
  s.idx.resize(n);
  for (size_t i = 0; i < n; ++i) {
    int64_t p = pos[o.b[i]]++;
    s.cam[p] = o.a[i];
    s.idx[p] = (int32_t)i;
  }
  for (int f = 0; f < nfeat; ++f) {
    std::vector<std::pair<int32_t, int32_t>> v;
    for (int64_t p = s.off[f]; p < s.off[f + 1]; ++p) v.push_back({s.cam[p], s.idx[p]});
    std::sort(v.begin(), v.end());
    for (size_t k = 0; k < v.size(); ++k) {
      if (k && v[k].first == v[k - 1].first)
        throw BaError(BA_E_INVALID, std::string("duplicate ") + what + " observation of feature " + std::to_string(f) +
                                        " in camera " + std::to_string(v[k].first));
      s.cam[s.off[f] + k] = v[k].first;
      s.idx[s.off[f] + k] = v[k].second;
    }
  }
  return s;
}

// Dense solver tables (host).  Entries: one per (feature, distinct block of its
// records), in feature order (off2 / fb).  Pairs (a <= b): every diagonal pair, the block
// pairs of each feature, the (camera, plane) pairs of the plane-association records and
// the group pairs of the relations; numbered in (a, b) order.  Per pair, its feature
// entries in feature order, then its U entries in record order.
void build_dense_tables(ba_handle* h, const std::vector<Rec> (&R)[NFAM], const std::vector<int64_t>& off2,
                        const std::vector<int32_t>& fb) {
  auto& D = h->dense;
  const int nb = h->nc + h->ng + h->nv;
  const int nfeat = h->np + h->nl;
  if ((int64_t)fb.size() > INT32_MAX) {
    D.why = "too many (feature, block) entries for the dense solver";
    return;
  }
  std::vector<int32_t> pid((size_t)nb * nb, -1);
  auto at = [&](int a, int b) -> int32_t& { return a <= b ? pid[(size_t)a * nb + b] : pid[(size_t)b * nb + a]; };
  auto rel_block = [&](size_t i, bool second) {
    const int g = second ? h->rel_gb[i] : h->rel_ga[i];
    return h->rel_kind[i] >= 2 ? h->nc + g : h->nc + h->ng + g;
  };
  int64_t n_ent = 0;
  for (int b = 0; b < nb; ++b) at(b, b) = 0;
  for (int f = 0; f < nfeat; ++f)
    for (int64_t i = off2[f]; i < off2[f + 1]; ++i)
      for (int64_t j = i; j < off2[f + 1]; ++j) {
        at(fb[i], fb[j]) = 0;
        ++n_ent;
      }
  if (n_ent > INT32_MAX) {
    D.why = "too many shared-feature terms for the dense solver";
    return;
  }
  for (int fam = 3; fam <= 4; ++fam)
    for (const Rec& r : R[fam]) at(r.cam, h->nc + r.grp) = 0;
  for (size_t i = 0; i < h->rel_kind.size(); ++i) at(rel_block(i, false), rel_block(i, true)) = 0;
  D.pair_ab.clear();
  for (int a = 0; a < nb; ++a)
    for (int b = a; b < nb; ++b) {
      int32_t& p = pid[(size_t)a * nb + b];
      if (p == 0) {
        p = (int32_t)D.pair_ab.size();
        D.pair_ab.push_back(make_int2(a, b));
      }
    }
  const size_t np_ = D.pair_ab.size();
  D.pair_off.assign(np_ + 1, 0);
  D.pair_uoff.assign(np_ + 1, 0);
  for (int f = 0; f < nfeat; ++f)
    for (int64_t i = off2[f]; i < off2[f + 1]; ++i)
      for (int64_t j = i; j < off2[f + 1]; ++j) D.pair_off[at(fb[i], fb[j]) + 1]++;
  for (int fam = 3; fam <= 4; ++fam)
    for (const Rec& r : R[fam]) D.pair_uoff[at(r.cam, h->nc + r.grp) + 1]++;
  for (size_t i = 0; i < h->rel_kind.size(); ++i) D.pair_uoff[at(rel_block(i, false), rel_block(i, true)) + 1]++;
  for (size_t p = 0; p < np_; ++p) {
    D.pair_off[p + 1] += D.pair_off[p];
    D.pair_uoff[p + 1] += D.pair_uoff[p];
  }
  D.pair_ent.assign((size_t)D.pair_off[np_], make_int2(0, 0));
  D.pair_u.assign((size_t)D.pair_uoff[np_], make_int2(0, 0));
  std::vector<int32_t> fill(D.pair_off.begin(), D.pair_off.end() - 1);
  for (int f = 0; f < nfeat; ++f)
    for (int64_t i = off2[f]; i < off2[f + 1]; ++i)
      for (int64_t j = i; j < off2[f + 1]; ++j)
        D.pair_ent[fill[at(fb[i], fb[j])]++] = make_int2((int)i, (int)j);
  fill.assign(D.pair_uoff.begin(), D.pair_uoff.end() - 1);
  for (int fam = 3; fam <= 4; ++fam)
    for (size_t k = 0; k < R[fam].size(); ++k) {
      const Rec& r = R[fam][k];
      D.pair_u[fill[at(r.cam, h->nc + r.grp)]++] = make_int2(fam, (int)k);
    }
  for (size_t i = 0; i < h->rel_kind.size(); ++i) {
    const int a = rel_block(i, false), b = rel_block(i, true);
    D.pair_u[fill[at(a, b)]++] = make_int2(a < b ? 8 : 9, (int)i);
  }
  // pairs with many shared features are summed in chunks
  D.chunk.clear();
  D.pair_choff.assign(np_ + 1, 0);
  for (size_t p = 0; p < np_; ++p) {
    const int32_t b = D.pair_off[p], e = D.pair_off[p + 1];
    if (e - b > DENSE_CHUNK)
      for (int32_t c = b; c < e; c += DENSE_CHUNK) D.chunk.push_back(make_int2(c, std::min(e, c + DENSE_CHUNK)));
    D.pair_choff[p + 1] = (int32_t)D.chunk.size();
  }
  D.fent.resize(fb.size());
  for (int f = 0; f < nfeat; ++f)
    for (int64_t i = off2[f]; i < off2[f + 1]; ++i) D.fent[i] = make_int2(f, fb[i]);
  D.built = true;
  D.why.clear();
}

// device storage of the dense solver, allocated and filled on first use
void dense_prepare(ba_handle* h) {
  auto& D = h->dense;
  if (!D.built) throw BaError(BA_E_INVALID, "dense solver unavailable: " + D.why);
  if (D.uploaded) return;
  Dev& d = h->d;
  DevAlloc& A = h->alloc;
  d.dense_n = d.nA;
  d.dense_npad = (d.nA + DENSE_NB - 1) / DENSE_NB * DENSE_NB;
  d.n_fent = (int)D.fent.size();
  d.n_pair = (int)D.pair_ab.size();
  d.n_chunk = (int)D.chunk.size();
  if (d.nA > 0) {
    d.chunk = A.get<int2>(D.chunk.size());
    d.pair_choff = A.get<int32_t>(D.pair_choff.size());
    d.dpart = A.get<double>((size_t)3 * 64 * D.chunk.size());
    upload(h, d.chunk, D.chunk);
    upload(h, d.pair_choff, D.pair_choff);
    d.fent = A.get<int2>(D.fent.size());
    d.pair_ab = A.get<int2>(D.pair_ab.size());
    d.pair_ent = A.get<int2>(D.pair_ent.size());
    d.pair_u = A.get<int2>(D.pair_u.size());
    d.pair_off = A.get<int32_t>(D.pair_off.size());
    d.pair_uoff = A.get<int32_t>(D.pair_uoff.size());
    d.dY = A.get<double>((size_t)DENSE_Y * D.fent.size());
    d.dS = A.get<double>((size_t)d.dense_npad * d.dense_npad);
    d.dLinv = A.get<double>((size_t)d.dense_npad * DENSE_NB);
    d.dv = A.get<double>(d.dense_npad);
    d.dw = A.get<double>(d.dense_npad);
    upload(h, d.fent, D.fent);
    upload(h, d.pair_ab, D.pair_ab);
    upload(h, d.pair_ent, D.pair_ent);
    upload(h, d.pair_u, D.pair_u);
    upload(h, d.pair_off, D.pair_off);
    upload(h, d.pair_uoff, D.pair_uoff);
  }
  d.dinfo = A.get<int>(1);
  sync(h);
  D.uploaded = true;
}

// the direct solve of S h_a = b for the current lambda into d.x; false when S is
// not positive definite (d.x unchanged)
bool dense_solve(ba_handle* h, double lambda) {
  dense_prepare(h);
  launch_dense_solve(h->d, lambda, h->stream);
  check_launch("dense solve");
  int info = 0;
  HIPCHK(hipMemcpyAsync(&info, h->d.dinfo, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  sync(h);
  return info == 0;
}

void finalize(ba_handle* h) {
  set_device(h);
  const Obs& OP = h->obs[BA_OBS_POINT];
  const Obs& OL = h->obs[BA_OBS_LINE];
  CSR P = build_csr(OP, h->np, "point");
  CSR L = build_csr(OL, h->nl, "line");

  // group memberships: at most one plane per feature, one VP per line
  std::vector<int32_t> pt_plane(h->np, -1), ln_plane(h->nl, -1), ln_vp(h->nl, -1);
  {
    const Obs& o = h->obs[BA_ASSOC_PLANE_POINT];
    for (size_t i = 0; i < o.a.size(); ++i) {
      if (pt_plane[o.b[i]] >= 0) throw BaError(BA_E_INVALID, "point " + std::to_string(o.b[i]) + " is associated with two planes");
      pt_plane[o.b[i]] = o.a[i];
    }
    const Obs& o2 = h->obs[BA_ASSOC_PLANE_LINE];
    for (size_t i = 0; i < o2.a.size(); ++i) {
      if (ln_plane[o2.b[i]] >= 0) throw BaError(BA_E_INVALID, "line " + std::to_string(o2.b[i]) + " is associated with two planes");
      ln_plane[o2.b[i]] = o2.a[i];
    }
    const Obs& o3 = h->obs[BA_ASSOC_VP_LINE];
    for (size_t i = 0; i < o3.a.size(); ++i) {
      if (ln_vp[o3.b[i]] >= 0) throw BaError(BA_E_INVALID, "line " + std::to_string(o3.b[i]) + " is associated with two VPs");
      ln_vp[o3.b[i]] = o3.a[i];
    }
  }
  // surface groups: at most one shape per point, one cuboid per line
  std::vector<int32_t> pt_shape(h->np, -1), ln_shape(h->nl, -1);
  {
    const Obs& o = h->obs[BA_ASSOC_SHAPE_POINT];
    for (size_t i = 0; i < o.a.size(); ++i) {
      if (pt_shape[o.b[i]] >= 0) throw BaError(BA_E_INVALID, "point " + std::to_string(o.b[i]) + " is on two shapes");
      pt_shape[o.b[i]] = o.a[i];
    }
    const Obs& o2 = h->obs[BA_ASSOC_SHAPE_LINE];
    for (size_t i = 0; i < o2.a.size(); ++i) {
      if (ln_shape[o2.b[i]] >= 0) throw BaError(BA_E_INVALID, "line " + std::to_string(o2.b[i]) + " is on two shapes");
      if ((int)h->sh[(size_t)SH_STRIDE * o2.a[i] + 15] != SH_CUBOID)
        throw BaError(BA_E_INVALID, "shape " + std::to_string(o2.a[i]) + " constrains lines but is not a cuboid");
      ln_shape[o2.b[i]] = o2.a[i];
    }
  }
  // junctions, deduplicated check
  const Obs& OJ = h->obs[BA_ASSOC_JUNCTION];
  {
    std::vector<int64_t> jk(OJ.a.size());
    for (size_t i = 0; i < OJ.a.size(); ++i) jk[i] = (int64_t)OJ.a[i] * h->nl + OJ.b[i];
    std::sort(jk.begin(), jk.end());
    if (std::adjacent_find(jk.begin(), jk.end()) != jk.end()) throw BaError(BA_E_INVALID, "duplicate junction");
  }

  // per-feature record counts for the signature ordering
  std::vector<int32_t> n6(h->np, 0), n7(h->nl, 0);
  for (size_t i = 0; i < OJ.a.size(); ++i) {
    const int j = OJ.a[i], k = OJ.b[i];
    for (int64_t p = L.off[k]; p < L.off[k + 1]; ++p) if (!P.has(j, L.cam[p])) n6[j]++;
    for (int64_t p = P.off[j]; p < P.off[j + 1]; ++p) if (!L.has(k, P.cam[p])) n7[k]++;
  }
  // internal order: features sorted by where their observing cameras are (so that a run
  // of consecutive features touches few cameras: the product keeps a workgroup's entries
  // of the reduced vector in LDS), then by record signature
  h->pt_perm.resize(h->np);
  std::iota(h->pt_perm.begin(), h->pt_perm.end(), 0);
  auto ptkey = [&](int j) {
    const int n1 = (int)(P.off[j + 1] - P.off[j]);
    return std::make_tuple(pt_plane[j] >= 0 && n1 > 0, n6[j] > 0, n1, n6[j]);
  };
  // locality key: Morton code of the mean centre of the feature's observing cameras
  std::vector<double> ctr((size_t)3 * h->nc);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int i = 0; i < h->nc; ++i) {
    const double* c = &h->cam[(size_t)CAM_STRIDE * i];
    for (int k = 0; k < 3; ++k) {
      const double v = -(c[k] * c[9] + c[3 + k] * c[10] + c[6 + k] * c[11]);
      ctr[3 * i + k] = v;
      lo[k] = std::min(lo[k], v);
      hi[k] = std::max(hi[k], v);
    }
  }
  // per-camera passes: cameras in Morton order of their centres, dealt to the XCDs in
  // contiguous runs (workgroup b runs on XCD b mod CU_XCDS)
  std::vector<int32_t> cam_wg(h->nc);
  {
    constexpr int CU_XCDS = 8;
    std::vector<uint64_t> ckey(h->nc);
    for (int i = 0; i < h->nc; ++i) {
      uint32_t q[3];
      for (int k = 0; k < 3; ++k) {
        const double span = hi[k] - lo[k];
        const double u = span > 0 ? (ctr[3 * i + k] - lo[k]) / span : 0.0;
        q[k] = (uint32_t)std::min(1023.0, std::max(0.0, u * 1024.0));
      }
      uint64_t code = 0;
      for (int bit = 9; bit >= 0; --bit)
        for (int k = 0; k < 3; ++k) code = (code << 1) | ((q[k] >> bit) & 1u);
      ckey[i] = code;
    }
    std::vector<int32_t> sorted(h->nc);
    std::iota(sorted.begin(), sorted.end(), 0);
    std::stable_sort(sorted.begin(), sorted.end(), [&](int a, int b) { return ckey[a] < ckey[b]; });
    const int chunk = (h->nc + CU_XCDS - 1) / CU_XCDS;
    std::vector<int> next(CU_XCDS);
    for (int x = 0; x < CU_XCDS; ++x) next[x] = x * chunk;
    for (int b = 0; b < h->nc; ++b) {
      const int x = b % CU_XCDS;
      cam_wg[b] = next[x] < std::min((x + 1) * chunk, h->nc) ? sorted[next[x]++] : -1;
    }
    // a workgroup whose XCD's run is used up takes a camera not dealt out, in order
    std::vector<char> used(h->nc, 0);
    for (int b = 0; b < h->nc; ++b)
      if (cam_wg[b] >= 0) used[cam_wg[b]] = 1;
    int r = 0;
    for (int b = 0; b < h->nc; ++b)
      if (cam_wg[b] < 0) {
        while (used[sorted[r]]) ++r;
        cam_wg[b] = sorted[r];
        used[sorted[r]] = 1;
      }
    for (int i = 0; i < h->nc; ++i)
      if (!used[i]) throw BaError(BA_E_STATE, "camera order is not a permutation");
  }
  auto morton = [&](const CSR& O, int f) -> uint64_t {
    const int64_t b = O.off[f], e = O.off[f + 1];
    if (e == b) return ~0ull;
    double m[3] = {0, 0, 0};
    for (int64_t p = b; p < e; ++p)
      for (int k = 0; k < 3; ++k) m[k] += ctr[3 * (size_t)O.cam[p] + k];
    uint64_t code = 0;
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
      const double span = hi[k] - lo[k];
      const double u = span > 0 ? (m[k] / (double)(e - b) - lo[k]) / span : 0.0;
      q[k] = (uint32_t)std::min(1023.0, std::max(0.0, u * 1024.0));
    }
    for (int bit = 9; bit >= 0; --bit)
      for (int k = 0; k < 3; ++k) code = (code << 1) | ((q[k] >> bit) & 1u);
    return code;
  };
  {
    std::vector<uint64_t> key(h->np);
    for (int j = 0; j < h->np; ++j) key[j] = morton(P, j);
    std::stable_sort(h->pt_perm.begin(), h->pt_perm.end(), [&](int a, int b) {
      return key[a] != key[b] ? key[a] < key[b] : ptkey(a) > ptkey(b);
    });
  }
  h->ln_perm.resize(h->nl);
  std::iota(h->ln_perm.begin(), h->ln_perm.end(), 0);
  auto lnkey = [&](int k) {
    const int n2 = (int)(L.off[k + 1] - L.off[k]);
    return std::make_tuple(ln_plane[k] >= 0 && n2 > 0, ln_vp[k] >= 0, n7[k] > 0, n2, n7[k]);
  };
  {
    std::vector<uint64_t> key(h->nl);
    for (int k = 0; k < h->nl; ++k) key[k] = morton(L, k);
    std::stable_sort(h->ln_perm.begin(), h->ln_perm.end(), [&](int a, int b) {
      return key[a] != key[b] ? key[a] < key[b] : lnkey(a) > lnkey(b);
    });
  }
  h->pt_inv.assign(h->np, 0);
  h->ln_inv.assign(h->nl, 0);
  for (int i = 0; i < h->np; ++i) h->pt_inv[h->pt_perm[i]] = i;
  for (int i = 0; i < h->nl; ++i) h->ln_inv[h->ln_perm[i]] = i;

  const double cx = h->cx, cy = h->cy;
  std::vector<Rec> R[NFAM];
  // R1: point observations;  R3: plane-point association x observing views
  for (int j = 0; j < h->np; ++j) {
    for (int64_t p = P.off[j]; p < P.off[j + 1]; ++p) {
      const int o = P.idx[p];
      const double* m = &OP.meas[4 * (size_t)o];
      Rec r{h->pt_inv[j], P.cam[p], -1, -1, {m[0] - cx, m[1] - cy, 0, 0}, {P.cam[p], j, -1}};
      R[1].push_back(r);
      if (pt_plane[j] >= 0) {
        Rec r3{h->pt_inv[j], P.cam[p], pt_plane[j], pt_plane[j], {0, 0, 0, 0}, {P.cam[p], j, pt_plane[j]}};
        R[3].push_back(r3);
      }
      if (pt_shape[j] >= 0) {  // family 9 (exported 13): the shape's projection, as R3
        Rec r9{h->pt_inv[j], P.cam[p], pt_shape[j], pt_shape[j], {0, 0, 0, 0}, {P.cam[p], j, pt_shape[j]}};
        R[9].push_back(r9);
      }
    }
  }
  // R2: line observations;  R4: plane-line association x observing views;  R5: VP-line
  for (int k = 0; k < h->nl; ++k) {
    for (int64_t p = L.off[k]; p < L.off[k + 1]; ++p) {
      const int o = L.idx[p];
      const double* m = &OL.meas[4 * (size_t)o];
      Rec r{h->ln_inv[k], L.cam[p], -1, -1, {m[0] - cx, m[1] - cy, m[2] - cx, m[3] - cy}, {L.cam[p], k, -1}};
      R[2].push_back(r);
      if (ln_plane[k] >= 0) {
        Rec r4 = r;
        r4.other = r4.grp = ln_plane[k];
        r4.key[2] = ln_plane[k];
        R[4].push_back(r4);
      }
      if (ln_shape[k] >= 0) {  // family 10 (exported 14): the cuboid face's plane projection, as R4
        Rec r10 = r;
        r10.other = r10.grp = ln_shape[k];
        r10.key[2] = ln_shape[k];
        R[10].push_back(r10);
      }
    }
    if (ln_vp[k] >= 0) {
      Rec r5{h->ln_inv[k], -1, ln_vp[k], ln_vp[k], {0, 0, 0, 0}, {-1, k, ln_vp[k]}};
      R[5].push_back(r5);
    }
  }
  // R6 / R7: cross-feature records over the views where exactly one feature is observed
  for (size_t i = 0; i < OJ.a.size(); ++i) {
    const int j = OJ.a[i], k = OJ.b[i];
    for (int64_t p = L.off[k]; p < L.off[k + 1]; ++p) {
      const int c = L.cam[p];
      if (P.has(j, c)) continue;
      const double* m = &OL.meas[4 * (size_t)L.idx[p]];
      // observed line through the two endpoints (shifted pixels), normalised
      const double a[3] = {m[0] - cx, m[1] - cy, 1.0}, b[3] = {m[2] - cx, m[3] - cy, 1.0};
      double l[3];
      cross(a, b, l);
      const double s = std::sqrt(l[0] * l[0] + l[1] * l[1]);
      if (!(s > 0)) throw BaError(BA_E_INVALID, "degenerate observed line segment");
      Rec r{h->pt_inv[j], c, k, -1, {l[0] / s, l[1] / s, l[2] / s, 0}, {c, j, k}};
      R[6].push_back(r);
    }
    for (int64_t p = P.off[j]; p < P.off[j + 1]; ++p) {
      const int c = P.cam[p];
      if (L.has(k, c)) continue;
      const double* m = &OP.meas[4 * (size_t)P.idx[p]];
      Rec r{h->ln_inv[k], c, j, -1, {m[2] - cx, m[3] - cy, 0, 0}, {c, k, j}};
      R[7].push_back(r);
    }
  }
  // family 8 (exported as 12): one record per 3D point-to-plane association, no camera
  {
    const Obs& o = h->obs[BA_ASSOC_PLANE_POINT_3D];
    std::vector<int64_t> pk(o.a.size());
    for (size_t i = 0; i < o.a.size(); ++i) pk[i] = (int64_t)o.b[i] * std::max(h->ng, 1) + o.a[i];
    std::sort(pk.begin(), pk.end());
    if (std::adjacent_find(pk.begin(), pk.end()) != pk.end())
      throw BaError(BA_E_INVALID, "duplicate 3D point-to-plane association");
    for (size_t i = 0; i < o.a.size(); ++i) {
      const int g = o.a[i], j = o.b[i];
      Rec r8{h->pt_inv[j], -1, g, g, {0, 0, 0, 0}, {-1, j, g}};
      R[8].push_back(r8);
    }
  }
  // feature-major order: (internal feature, camera, other)
  for (int fam = 1; fam < NFAM; ++fam)
    std::sort(R[fam].begin(), R[fam].end(), [](const Rec& a, const Rec& b) {
      if (a.feat != b.feat) return a.feat < b.feat;
      if (a.cam != b.cam) return a.cam < b.cam;
      return a.other < b.other;
    });

  // ---- device layout
  Dev& d = h->d;
  d.CD = h->CD; d.nc = h->nc; d.np = h->np; d.nl = h->nl; d.ng = h->ng; d.nv = h->nv; d.ns = h->ns;
  d.offPl = h->CD * h->nc;
  d.offVp = d.offPl + 3 * h->ng;
  d.offSh = d.offVp + 2 * h->nv;
  d.nA = d.offSh + SH_DOF * h->ns;
  d.fp64 = h->precision == BA_PREC_FP64 ? 1 : 0;
  const size_t TS = d.fp64 ? sizeof(double) : sizeof(float);
  DevAlloc& A = h->alloc;
  // parameters (internal feature order)
  std::vector<double> ptI((size_t)h->np * PT_STRIDE), lnI((size_t)h->nl * LN_STRIDE);
  for (int i = 0; i < h->np; ++i) std::copy_n(&h->pt[(size_t)PT_STRIDE * h->pt_perm[i]], PT_STRIDE, &ptI[(size_t)PT_STRIDE * i]);
  for (int i = 0; i < h->nl; ++i) std::copy_n(&h->ln[(size_t)LN_STRIDE * h->ln_perm[i]], LN_STRIDE, &lnI[(size_t)LN_STRIDE * i]);
  d.cam64 = A.get<double>(h->cam.size()); d.cam64n = A.get<double>(h->cam.size());
  d.pt64 = A.get<double>(ptI.size()); d.pt64n = A.get<double>(ptI.size());
  d.ln64 = A.get<double>(lnI.size()); d.ln64n = A.get<double>(lnI.size());
  d.pl64 = A.get<double>(h->pl.size()); d.pl64n = A.get<double>(h->pl.size());
  d.vp64 = A.get<double>(h->vp.size()); d.vp64n = A.get<double>(h->vp.size());
  upload(h, d.cam64, h->cam); upload(h, d.pt64, ptI); upload(h, d.ln64, lnI);
  upload(h, d.pl64, h->pl); upload(h, d.vp64, h->vp);
  d.sh64 = A.get<double>(h->sh.size()); d.sh64n = A.get<double>(h->sh.size());
  upload(h, d.sh64, h->sh);
  d.camT = A.get<char>(h->cam.size(), TS); d.ptT = A.get<char>(ptI.size(), TS); d.lnT = A.get<char>(lnI.size(), TS);
  d.plT = A.get<char>(h->pl.size(), TS); d.vpT = A.get<char>(h->vp.size(), TS);

  // families
  int64_t max_blocks = 0;
  std::vector<int32_t> foff_h[NFAM], fcam_h[NFAM], fgrp_h[NFAM];
  for (int fam = 1; fam < NFAM; ++fam) {
    const auto& v = R[fam];
    const int64_t n = (int64_t)v.size();
    d.fn[fam] = n;
    const int nfeat = fam_is_line(fam) ? h->nl : h->np;
    std::vector<int32_t> cam(n), grp(n), feat(n), off(nfeat + 1, 0);
    const int mw = meas_width(fam);
    std::vector<double> meas((size_t)n * mw);
    h->keys[fam].resize((size_t)n * 3);
    for (int64_t i = 0; i < n; ++i) {
      cam[i] = v[i].cam; grp[i] = v[i].grp; feat[i] = v[i].feat;
      off[v[i].feat + 1]++;
      for (int k = 0; k < mw; ++k) meas[(size_t)i * mw + k] = v[i].meas[k];
      for (int k = 0; k < 3; ++k) h->keys[fam][(size_t)i * 3 + k] = v[i].key[k];
    }
    for (int f = 0; f < nfeat; ++f) off[f + 1] += off[f];
    foff_h[fam] = off;
    fcam_h[fam] = cam;
    fgrp_h[fam] = grp;
    d.fcam[fam] = A.get<int32_t>(n); d.fgrp[fam] = A.get<int32_t>(n); d.ffeat[fam] = A.get<int32_t>(n);
    d.foff[fam] = A.get<int32_t>(nfeat + 1);
    d.fmeas[fam] = A.get<double>((size_t)n * std::max(mw, 1));
    d.frec[fam] = A.get<char>((size_t)n * slot_stride(fam, h->CD), TS);
    d.fres[fam] = A.get<char>((size_t)n * fam_rows(fam), TS);
    upload(h, d.fcam[fam], cam); upload(h, d.fgrp[fam], grp); upload(h, d.ffeat[fam], feat);
    upload(h, d.foff[fam], off); upload(h, d.fmeas[fam], meas);
    const int kind = fam == 1 ? BA_OBS_POINT : fam == 2 ? BA_OBS_LINE : fam == 3 ? BA_ASSOC_PLANE_POINT
                     : fam == 4 ? BA_ASSOC_PLANE_LINE : fam == 5 ? BA_ASSOC_VP_LINE
                     : fam == 8 ? BA_ASSOC_PLANE_POINT_3D : fam == 9 ? BA_ASSOC_SHAPE_POINT
                     : fam == 10 ? BA_ASSOC_SHAPE_LINE : BA_ASSOC_JUNCTION;
    const ba_loss lo = h->obs[kind].loss_set ? h->obs[kind].loss : default_loss(kind);
    d.lkind[fam] = lo.kind; d.lscale[fam] = lo.scale; d.lweight[fam] = lo.weight;
    max_blocks += (n + 255) / 256;
    if (n > INT32_MAX) throw BaError(BA_E_INVALID, "too many records in one family");
  }
  // inter-group relations: records, losses per kind, and per group block (planes, then
  // VPs) the CSR of its entries (2 * record + side)
  {
    h->rel_ga.clear(); h->rel_gb.clear(); h->rel_kind.clear();
    for (int k = 0; k < 4; ++k) {
      const Obs& o = h->obs[BA_REL_VP_ORTHO + k];
      const ba_loss lo = o.loss_set ? o.loss : default_loss(BA_REL_VP_ORTHO + k);
      d.rel_lkind[k] = lo.kind; d.rel_lscale[k] = lo.scale; d.rel_lweight[k] = lo.weight;
      for (size_t i = 0; i < o.a.size(); ++i) {
        h->rel_ga.push_back(o.a[i]); h->rel_gb.push_back(o.b[i]); h->rel_kind.push_back(k);
      }
    }
    const int n = (int)h->rel_kind.size();
    d.n_rel = n;
    const int nb = h->ng + h->nv;
    std::vector<int32_t> goff(nb + 1, 0), gent(2 * (size_t)n);
    auto block = [&](int i, int side) {
      const int g = side ? h->rel_gb[i] : h->rel_ga[i];
      return h->rel_kind[i] >= 2 ? g : h->ng + g;
    };
    for (int i = 0; i < n; ++i)
      for (int side = 0; side < 2; ++side) goff[block(i, side) + 1]++;
    for (int b = 0; b < nb; ++b) goff[b + 1] += goff[b];
    std::vector<int32_t> fill(goff.begin(), goff.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int side = 0; side < 2; ++side) gent[fill[block(i, side)]++] = 2 * i + side;
    d.rel_ga = A.get<int32_t>(n); d.rel_gb = A.get<int32_t>(n); d.rel_kind = A.get<int32_t>(n);
    d.rel_goff = A.get<int32_t>(nb + 1); d.rel_gent = A.get<int32_t>(2 * (size_t)n);
    d.rel_r = A.get<double>(3 * (size_t)n); d.rel_J = A.get<double>(18 * (size_t)n);
    d.rel_y = A.get<double>(d.nA);
    launch_zero(d.rel_y, (size_t)std::max(d.nA, 1) * sizeof(double), h->stream);
    upload(h, d.rel_ga, h->rel_ga); upload(h, d.rel_gb, h->rel_gb); upload(h, d.rel_kind, h->rel_kind);
    upload(h, d.rel_goff, goff); upload(h, d.rel_gent, gent);
    if (n) max_blocks += 1;  // one cost partial
  }
  // record mask (all clear)
  d.has_mask = 0;
  d.mpt = A.get<uint8_t>(h->np); d.mln = A.get<uint8_t>(h->nl);
  d.mpl = A.get<uint8_t>(h->ng); d.mvp = A.get<uint8_t>(h->nv);
  launch_zero(d.mpt, std::max(h->np, 1), h->stream); launch_zero(d.mln, std::max(h->nl, 1), h->stream);
  launch_zero(d.mpl, std::max(h->ng, 1), h->stream); launch_zero(d.mvp, std::max(h->nv, 1), h->stream);
  // block graph of the reduced system (blocks are adjacent when they share a feature)
  // and the dense solver's tables
  {
    const int nblocks = h->nc + h->ng + h->nv;
    const bool want_graph = nblocks > 0 && nblocks <= ba_gnn_impl::MAX_GRAPH_NODES;
    const bool want_dense = d.nA > 0 && d.nA <= DENSE_MAX_NA && h->ns == 0;
    h->dense = ba_handle::DenseHost();
    if (h->ns > 0) h->dense.why = "the dense solver does not take surface groups (shapes)";
    else if (d.nA > DENSE_MAX_NA)
      h->dense.why = "the reduced system has " + std::to_string(d.nA) + " rows, more than the dense solver's " +
                     std::to_string(DENSE_MAX_NA);
    if (d.nA == 0) {
      h->dense.built = true;
      h->dense.why.clear();
    }
    if (want_graph || want_dense) {
      const int nfeat = h->np + h->nl;
      std::vector<int64_t> fb_off(nfeat + 1, 0), block_records(nblocks, 0);
      // blocks of cameras, planes and VPs (the network's graph has no shape nodes)
      auto block_of = [&](int fam, const Rec& r, int32_t out[2]) {
        int k = 0;
        if (r.cam >= 0) out[k++] = r.cam;
        if (r.grp >= 0 && fam != 9 && fam != 10) out[k++] = (fam == 5 ? h->nc + h->ng : h->nc) + r.grp;
        return k;
      };
      auto fid = [&](int fam, const Rec& r) { return fam_is_line(fam) ? h->np + r.feat : r.feat; };
      for (int fam = 1; fam < NFAM; ++fam)
        for (const Rec& r : R[fam]) {
          int32_t b[2];
          const int k = block_of(fam, r, b);
          fb_off[fid(fam, r) + 1] += k;
          for (int q = 0; q < k; ++q) block_records[b[q]]++;
        }
      for (int f = 0; f < nfeat; ++f) fb_off[f + 1] += fb_off[f];
      std::vector<int32_t> fb(fb_off[nfeat]);
      std::vector<int64_t> fill(fb_off.begin(), fb_off.end() - 1);
      for (int fam = 1; fam < NFAM; ++fam)
        for (const Rec& r : R[fam]) {
          int32_t b[2];
          const int k = block_of(fam, r, b);
          for (int q = 0; q < k; ++q) fb[fill[fid(fam, r)]++] = b[q];
        }
      // distinct blocks per feature, compacted in place
      std::vector<int64_t> off2(nfeat + 1, 0);
      int64_t w = 0;
      for (int f = 0; f < nfeat; ++f) {
        auto b = fb.begin() + fb_off[f], e = fb.begin() + fb_off[f + 1];
        std::sort(b, e);
        e = std::unique(b, e);
        for (auto it = b; it != e; ++it) fb[w++] = *it;
        off2[f + 1] = w;
      }
      fb.resize(w);
      // scene scale: RMS distance of the input camera centres -R^T t from their mean
      double s0 = 0, mean[3] = {0, 0, 0};
      std::vector<double> ctr((size_t)3 * h->nc);
      for (int i = 0; i < h->nc; ++i) {
        const double* c = &h->cam[(size_t)CAM_STRIDE * i];
        for (int k = 0; k < 3; ++k) {
          ctr[3 * i + k] = -(c[k] * c[9] + c[3 + k] * c[10] + c[6 + k] * c[11]);
          mean[k] += ctr[3 * i + k] / h->nc;
        }
      }
      for (int i = 0; i < h->nc; ++i)
        for (int k = 0; k < 3; ++k) s0 += (ctr[3 * i + k] - mean[k]) * (ctr[3 * i + k] - mean[k]) / h->nc;
      s0 = std::sqrt(s0);
      if (!(s0 > 0) || !std::isfinite(s0)) s0 = 1.0;
      if (want_graph) ba_gnn_impl::build_graph(h->graph, h->nc, h->ng, h->nv, h->CD, off2, fb, block_records, s0);
      if (want_dense) build_dense_tables(h, R, off2, fb);
    }
    if (h->graph.valid) {
      const auto& G = h->graph;
      h->g_stat = A.get<float>(G.node_static.size());
      h->g_type = A.get<int32_t>(G.n_nodes);
      h->g_x = A.get<float>(G.node_static.size());
      upload(h, h->g_stat, G.node_static);
      upload(h, h->g_type, G.node_type);
    }
  }
  // camera-major lists
  auto cam_major = [&](int fam, bool runs, int32_t*& idx_or_start, int32_t*& cnt, int32_t*& off) {
    const auto& v = R[fam];
    std::vector<std::vector<int32_t>> bucket(h->nc), bcnt(h->nc);
    for (size_t i = 0; i < v.size();) {
      size_t j = i + 1;
      if (runs)
        while (j < v.size() && v[j].feat == v[i].feat && v[j].cam == v[i].cam) ++j;
      bucket[v[i].cam].push_back((int32_t)i);
      bcnt[v[i].cam].push_back((int32_t)(j - i));
      i = j;
    }
    std::vector<int32_t> o(h->nc + 1, 0), flat, fc;
    for (int c = 0; c < h->nc; ++c) {
      o[c + 1] = o[c] + (int32_t)bucket[c].size();
      flat.insert(flat.end(), bucket[c].begin(), bucket[c].end());
      fc.insert(fc.end(), bcnt[c].begin(), bcnt[c].end());
    }
    idx_or_start = A.get<int32_t>(flat.size());
    off = A.get<int32_t>(o.size());
    upload(h, idx_or_start, flat);
    upload(h, off, o);
    if (runs) {
      cnt = A.get<int32_t>(fc.size());
      upload(h, cnt, fc);
    }
  };
  // per camera, the range of its observations in the camera-major copies below
  auto cam_offsets = [&](int fam, int32_t*& off) {
    std::vector<int32_t> o(h->nc + 1, 0);
    for (const auto& rec : R[fam]) o[rec.cam + 1]++;
    for (int c = 0; c < h->nc; ++c) o[c + 1] += o[c];
    off = A.get<int32_t>(o.size());
    upload(h, off, o);
  };
  d.cam_order = A.get<int32_t>(std::max(h->nc, 1));
  upload(h, d.cam_order, cam_wg);
  cam_offsets(1, d.po_off);
  cam_offsets(2, d.lo_off);
  // camera-major copies of the observation slots and their aligned plane slots
  for (int pair = 0; pair < 2; ++pair) {
    const int fo = pair == 0 ? 1 : 2, fp = pair == 0 ? 3 : 4;
    const auto& v = R[fo];
    if (v.empty()) continue;
    std::vector<std::vector<int32_t>> bucket(h->nc);
    for (size_t i = 0; i < v.size(); ++i) bucket[v[i].cam].push_back((int32_t)i);
    const int64_t n = (int64_t)v.size(), np_ = (int64_t)R[fp].size();
    std::vector<int32_t> pos(n), feat(n), al(n, -1), ppos(np_, -1), pgrp;
    int64_t j = 0, k = 0;
    for (int c = 0; c < h->nc; ++c)
      for (int32_t i : bucket[c]) {
        pos[i] = (int32_t)j;
        feat[j] = v[i].feat;
        const int f = v[i].feat;
        if (np_ && foff_h[fp][f + 1] > foff_h[fp][f]) {  // the point / line is in a plane
          const int64_t ip = foff_h[fp][f] + (i - foff_h[fo][f]);
          ppos[ip] = (int32_t)k;
          al[j] = (int32_t)k;
          pgrp.push_back(R[fp][ip].grp);
          ++k;
        }
        ++j;
      }
    d.cmrec[fo] = A.get<char>((size_t)n * slot_stride(fo, h->CD), TS);
    d.cmres[fo] = A.get<char>((size_t)n * fam_rows(fo), TS);
    d.cmpos[fo] = A.get<int32_t>(n); d.cmfeat[fo] = A.get<int32_t>(n); d.cmal[fo] = A.get<int32_t>(n);
    upload(h, d.cmpos[fo], pos); upload(h, d.cmfeat[fo], feat); upload(h, d.cmal[fo], al);
    if (np_) {
      if (k != np_) throw BaError(BA_E_INVALID, "plane records are not aligned with their observations");
      d.cmrec[fp] = A.get<char>((size_t)np_ * slot_stride(fp, h->CD), TS);
      d.cmres[fp] = A.get<char>((size_t)np_ * fam_rows(fp), TS);
      d.cmpos[fp] = A.get<int32_t>(np_); d.cmgrp[fp] = A.get<int32_t>(np_);
      upload(h, d.cmpos[fp], ppos); upload(h, d.cmgrp[fp], pgrp);
    }
  }
  // per R1 / R2 camera-major position, the family 9 / 10 record of the same feature and
  // camera (a feature's shape records follow its observations one to one)
  for (int pair = 0; pair < 2; ++pair) {
    const int fo = pair == 0 ? 1 : 2, fs = pair == 0 ? 9 : 10;
    if (R[fs].empty()) continue;
    const auto& v = R[fo];
    std::vector<int32_t> cmo(h->nc + 1, 0);
    for (const Rec& r : v) cmo[r.cam + 1]++;
    for (int c = 0; c < h->nc; ++c) cmo[c + 1] += cmo[c];
    std::vector<int32_t> al(v.size(), -1);
    int64_t matched = 0;
    for (size_t i = 0; i < v.size(); ++i) {
      const int f = v[i].feat;
      const int32_t pos = cmo[v[i].cam]++;
      if (foff_h[fs][f + 1] > foff_h[fs][f]) {
        const int64_t is = foff_h[fs][f] + ((int64_t)i - foff_h[fo][f]);
        if (R[fs][is].cam != v[i].cam) throw BaError(BA_E_STATE, "shape records are not aligned with their observations");
        al[pos] = (int32_t)is;
        ++matched;
      }
    }
    if (matched != (int64_t)R[fs].size()) throw BaError(BA_E_STATE, "shape records are not aligned with their observations");
    int32_t*& dst = pair == 0 ? d.shal_p : d.shal_l;
    dst = A.get<int32_t>(al.size());
    upload(h, dst, al);
    // the same records listed per camera, with their features
    std::vector<int32_t> cnt(h->nc + 1, 0), off(h->nc + 1, 0), rec, feat;
    for (const Rec& r : v) cnt[r.cam + 1]++;
    for (int c = 0; c < h->nc; ++c) cnt[c + 1] += cnt[c];
    for (int c = 0; c < h->nc; ++c) {
      for (int32_t pos = cnt[c]; pos < cnt[c + 1]; ++pos)
        if (al[pos] >= 0) {
          rec.push_back(al[pos]);
          feat.push_back(R[fs][al[pos]].feat);
        }
      off[c + 1] = (int32_t)rec.size();
    }
    d.shc_off[pair] = A.get<int32_t>(off.size());
    d.shc_rec[pair] = A.get<int32_t>(rec.size());
    d.shc_feat[pair] = A.get<int32_t>(feat.size());
    upload(h, d.shc_off[pair], off);
    upload(h, d.shc_rec[pair], rec);
    upload(h, d.shc_feat[pair], feat);
  }
  {
    std::vector<std::vector<int32_t>> mp(h->ns), ml(h->ns);
    for (size_t i = 0; i < R[9].size(); ++i)
      if (i == 0 || R[9][i].feat != R[9][i - 1].feat) mp[R[9][i].grp].push_back(R[9][i].feat);
    for (size_t i = 0; i < R[10].size(); ++i)
      if (i == 0 || R[10][i].feat != R[10][i - 1].feat) ml[R[10][i].grp].push_back(R[10][i].feat);
    auto flatten = [&](std::vector<std::vector<int32_t>>& m, int32_t*& list, int32_t*& off) {
      std::vector<int32_t> o(m.size() + 1, 0), flat;
      for (size_t g = 0; g < m.size(); ++g) {
        o[g + 1] = o[g] + (int32_t)m[g].size();
        flat.insert(flat.end(), m[g].begin(), m[g].end());
      }
      list = A.get<int32_t>(flat.size());
      off = A.get<int32_t>(o.size());
      upload(h, list, flat);
      upload(h, off, o);
    };
    flatten(mp, d.shp, d.shp_off);
    flatten(ml, d.shl, d.shl_off);
    // chunks of at most SH_CHUNK members of one shape for the shape passes
    std::vector<int4> ch;
    for (int kind = 0; kind < 2; ++kind) {
      int32_t o = 0;
      for (int q = 0; q < h->ns; ++q) {
        const int32_t n = (int32_t)(kind == 0 ? mp[q].size() : ml[q].size());
        for (int32_t c = 0; c < n; c += SH_CHUNK) ch.push_back(make_int4(q, o + c, std::min(SH_CHUNK, n - c), kind));
        o += n;
      }
    }
    d.n_shch = (int)ch.size();
    d.shch = A.get<int4>(ch.size());
    upload(h, d.shch, ch);
    d.shacc = A.get<double>((size_t)h->ns * SH_ACC);
    d.shsz = A.get<double>((size_t)h->ns * SH_DOF * SZ_COLS * SZ_PANELS);
  }
  cam_major(6, true, d.px_start, d.px_cnt, d.px_off);
  cam_major(7, true, d.lx_start, d.lx_cnt, d.lx_off);
  // group member lists
  {
    std::vector<std::vector<int32_t>> mp(h->ng), ml(h->ng), mv(h->nv);
    // points of a plane: through its plane-association records (R3) or its 3D
    // point-to-plane records (family 8), each point once, in feature order
    {
      std::vector<std::pair<int32_t, int32_t>> gp;
      for (const Rec& r : R[3]) gp.emplace_back(r.grp, r.feat);
      for (const Rec& r : R[8]) gp.emplace_back(r.grp, r.feat);
      std::sort(gp.begin(), gp.end());
      gp.erase(std::unique(gp.begin(), gp.end()), gp.end());
      for (auto [g, f] : gp) mp[g].push_back(f);
    }
    for (size_t i = 0; i < R[4].size(); ++i)
      if (i == 0 || R[4][i].feat != R[4][i - 1].feat) ml[R[4][i].grp].push_back(R[4][i].feat);
    for (size_t i = 0; i < R[5].size(); ++i) mv[R[5][i].grp].push_back((int32_t)i);
    auto flatten = [&](std::vector<std::vector<int32_t>>& m, int32_t*& list, int32_t*& off) {
      std::vector<int32_t> o(m.size() + 1, 0), flat;
      for (size_t g = 0; g < m.size(); ++g) {
        o[g + 1] = o[g] + (int32_t)m[g].size();
        flat.insert(flat.end(), m[g].begin(), m[g].end());
      }
      list = A.get<int32_t>(flat.size());
      off = A.get<int32_t>(o.size());
      upload(h, list, flat);
      upload(h, off, o);
    };
    flatten(mp, d.plp, d.plp_off);
    flatten(ml, d.pll, d.pll_off);
    flatten(mv, d.vpm, d.vpm_off);
  }
  // feature blocks
  d.Vp = A.get<char>((size_t)h->np * 6, TS); d.gp = A.get<char>((size_t)h->np * 3, TS);
  d.Vl = A.get<char>((size_t)h->nl * 10, TS); d.gl = A.get<char>((size_t)h->nl * 4, TS);
  d.Vip = A.get<char>((size_t)h->np * 6, TS); d.Vil = A.get<char>((size_t)h->nl * 10, TS);
  d.sp = A.get<char>((size_t)h->np * 3, TS); d.sl = A.get<char>((size_t)h->nl * 4, TS);
  d.Vip64 = A.get<double>((size_t)h->np * 6); d.Vil64 = A.get<double>((size_t)h->nl * 10);
  d.flp = A.get<uint8_t>(h->np); d.fll = A.get<uint8_t>(h->nl);
  d.Dp = A.get<double>((size_t)h->np * 3); d.Dl = A.get<double>((size_t)h->nl * 4);
  d.hp = A.get<double>((size_t)h->np * 3); d.hl = A.get<double>((size_t)h->nl * 4);
  // A side
  const int CD = h->CD, nA = d.nA;
  d.Ucam = A.get<double>((size_t)h->nc * CD * CD); d.Upl = A.get<double>((size_t)h->ng * 9); d.Uvp = A.get<double>((size_t)h->nv * 4);
  d.Scam = A.get<double>((size_t)h->nc * CD * CD); d.Spl = A.get<double>((size_t)h->ng * 9); d.Svp = A.get<double>((size_t)h->nv * 4);
  d.Mcam = A.get<double>((size_t)h->nc * CD * CD); d.Mpl = A.get<double>((size_t)h->ng * 9); d.Mvp = A.get<double>((size_t)h->nv * 4);
  d.Ush = A.get<double>((size_t)h->ns * SH_DOF * SH_DOF); d.Ssh = A.get<double>((size_t)h->ns * SH_DOF * SH_DOF);
  d.Msh = A.get<double>((size_t)h->ns * SH_DOF * SH_DOF);
  d.gA = A.get<double>(nA); d.DA = A.get<double>(nA); d.bA = A.get<double>(nA);
  d.x = A.get<double>(nA); d.r = A.get<double>(nA); d.z = A.get<double>(nA); d.p = A.get<double>(nA); d.q = A.get<double>(nA);
  d.xT = A.get<char>(nA, TS);
  // coarse space of the two-level preconditioners
  d.Zc = A.get<double>((size_t)COARSE_K * nA);
  d.SZc = A.get<double>((size_t)COARSE_K * nA);
  // the network writes its columns on the rows of its graph's nodes only: the shape
  // rows of those columns stay zero
  launch_zero(d.Zc, (size_t)COARSE_K * std::max(nA, 1) * sizeof(double), h->stream);
  d.Einv = A.get<double>((size_t)COARSE_K * COARSE_K);
  d.Ztb = A.get<double>((size_t)COARSE_K + COARSE_K * COARSE_K);
  d.szr = A.get<char>((size_t)nA * SZ_COLS * SZ_PANELS, TS);
  d.szfp = A.get<char>((size_t)h->np * 3 * SZ_COLS * SZ_PANELS, TS);
  d.szfl = A.get<char>((size_t)h->nl * 4 * SZ_COLS * SZ_PANELS, TS);
  // product tiles: runs of consecutive features with at most MV_TILE records over
  // all their families, one slot per record in feature order: (family << 28 | record,
  // camera, group, feature - first feature of the tile)
  {
    std::vector<int4> tiles;
    std::vector<int4> wrec;
    std::vector<int32_t> bigp, bigl;
    // BA_TILE_RECORDS (1..64) lowers the record capacity of a tile; used by tests
    // to route features through the large-feature path
    int cap = MV_TILE;
    if (const char* e = std::getenv("BA_TILE_RECORDS")) cap = std::max(1, std::min(MV_TILE, std::atoi(e)));
    for (int fam = 1; fam < NFAM; ++fam)
      if (d.fn[fam] >= (int64_t)1 << 28) throw BaError(BA_E_INVALID, "more than 2^28 records in one family");
    // a line on a cuboid (family 10, whose slots exceed the tiles' register budget) is a
    // large feature (one wavefront each in k_mv_big); points on shapes (family 9) go in
    // the tiles
    auto build = [&](const std::vector<int>& fams, int nfeat, std::vector<int32_t>& big, int fam_big) {
      auto on_shape = [&](int f) { return fam_big > 0 && foff_h[fam_big][f + 1] > foff_h[fam_big][f]; };
      int f = 0;
      while (f < nfeat) {
        const int fb = f;
        int64_t cnt = 0;
        while (f < nfeat && !on_shape(f)) {
          int64_t n = 0;
          for (int fam : fams) n += foff_h[fam][f + 1] - foff_h[fam][f];
          if (cnt + n > cap) break;
          cnt += n;
          ++f;
        }
        if (f == fb) {  // one feature with more records than a tile holds, or on a shape
          big.push_back(f);
          ++f;
          continue;
        }
        if (cnt == 0) continue;  // features without records
        const int first = (int)wrec.size();
        for (int g = fb; g < f; ++g)
          for (int fam : fams)
            for (int64_t r = foff_h[fam][g]; r < foff_h[fam][g + 1]; ++r)
              wrec.push_back(make_int4((int)(((uint32_t)fam << 28) | (uint32_t)r), fcam_h[fam][r], fgrp_h[fam][r], g - fb));
        tiles.push_back(make_int4(first, (int)cnt, fb, 0));
      }
    };
    build({1, 3, 6, 8, 9}, h->np, bigp, -1);
    d.n_ptiles = (int)tiles.size();
    build({2, 4, 5, 7}, h->nl, bigl, 10);
    d.n_tiles = (int)tiles.size();
    d.n_bigp = (int)bigp.size();
    d.n_bigl = (int)bigl.size();
    d.tiles = A.get<int4>(tiles.size());
    d.wrec = A.get<int4>(wrec.size());
    d.bigp = A.get<int32_t>(bigp.size());
    d.bigl = A.get<int32_t>(bigl.size());
    upload(h, d.tiles, tiles);
    upload(h, d.wrec, wrec);
    upload(h, d.bigp, bigp);
    upload(h, d.bigl, bigl);
  }
  // the workgroup's copy of the reduced vector in LDS when it fits
  int ncu = 0;
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device));
  const int max_lds = matvec_max_lds_bytes();
  d.mv_stage = !d.fp64 && d.fn[9] > 0 ? 1 : 0;
  const size_t stage_bytes = d.mv_stage ? MV_STAGE_BYTES : 0;
  if (stage_bytes > (size_t)max_lds) throw BaError(BA_E_DEVICE, "the product's LDS staging does not fit a workgroup");
  d.mv_lds = (size_t)nA * 8 + stage_bytes <= (size_t)max_lds ? 1 : 0;
  // BA_PRODUCT_GLOBAL_Y=1 accumulates the product in global memory whatever n_A (the mode
  // of reduced systems too large for LDS); used by tests
  if (const char* e = std::getenv("BA_PRODUCT_GLOBAL_Y"))
    if (std::atoi(e) != 0) d.mv_lds = 0;
  const size_t lds_bytes = matvec_lds_bytes(d);
  const int wg_per_cu = (int)std::max<size_t>(1, std::min<size_t>(2, 163840 / std::max<size_t>(lds_bytes, 1)));
  const int64_t waves = d.n_tiles + (d.n_bigp + d.n_bigl + 63) / 64;
  d.n_mv_wg = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)ncu * wg_per_cu, (waves + MV_THREADS / 64 - 1) / (MV_THREADS / 64)));
  const size_t mv_rows = d.mv_lds ? (size_t)d.n_mv_wg : 1;
  d.mv_part = A.get<double>(mv_rows * nA);
  d.cnt = A.get<unsigned int>(4);
  launch_zero(d.cnt, 4 * sizeof(unsigned int), h->stream);
  d.part2 = A.get<double>(2 * ((size_t)nA / 64 + 2) + 256);
  // deterministic mode: per-workgroup partials of every accumulator (the widest PCG
  // kernel has one workgroup per 64 entries) and the product's s_f
  d.det_stride = (int)std::max<int64_t>(1, ((int64_t)nA + 63) / 64);
  d.detp = A.get<double>((size_t)(SC_COUNT + COARSE_K) * d.det_stride);
  launch_zero(d.detp, (size_t)(SC_COUNT + COARSE_K) * d.det_stride * sizeof(double), h->stream);
  d.sdp = A.get<char>((size_t)h->np * 3, TS);
  d.sdl = A.get<char>((size_t)h->nl * 4, TS);
  launch_zero(d.mv_part, mv_rows * nA * sizeof(double), h->stream);
  d.scal = A.get<double>(SC_COUNT);
  launch_zero(d.scal, SC_COUNT * sizeof(double), h->stream);
  const int64_t fe_blocks = (h->np + 255) / 256 + (h->nl + 255) / 256;
  d.n_red_max = std::max<int64_t>(std::max(max_blocks, fe_blocks), 32);
  d.red = A.get<double>((size_t)(2 * d.n_red_max));
  HIPCHK(hipHostMalloc((void**)&h->hscal, SC_COUNT * sizeof(double), hipHostMallocDefault));
  if (h->gnn) ba_gnn_impl::attach(h->gnn, h->graph);
  check_launch("finalize");
  sync(h);
  h->finalized = true;
  if (std::getenv("BA_VERBOSE")) {
    std::fprintf(stderr, "[libba] records:");
    for (int fam = 1; fam < NFAM; ++fam) std::fprintf(stderr, " R%d=%lld", fam, (long long)d.fn[fam]);
    std::fprintf(stderr, "; nA=%d; product: %s, %d workgroups, %d tiles (%d point), %d+%d large features, LDS %zu of %d B\n",
                 nA, d.mv_lds ? "LDS-private y" : "global atomics", d.n_mv_wg, d.n_tiles,
                 d.n_ptiles, d.n_bigp, d.n_bigl, lds_bytes, max_lds);
  }
  h->need_lin = true;
}

void read_scal(ba_handle* h) {
  HIPCHK(hipMemcpyAsync(h->hscal, h->d.scal, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  sync(h);
}

void linearize_all(ba_handle* h) {
  launch_zero(h->d.scal + SC_NDEG, sizeof(double), h->stream);
  launch_cast_params(h->d, false, h->stream);
  launch_linearize(h->d, h->stream);
  launch_feature_accum(h->d, h->stream);
  launch_camera_pass_a(h->d, h->stream);
  launch_grad_inf(h->d, h->stream);
  check_launch("linearize");
  h->need_lin = false;
}

// damped feature inverses, b_a and the diagonal blocks of S
void assemble_schur(ba_handle* h, double lambda, double kappa_max) {
  launch_zero(h->d.scal + SC_NFLAG, sizeof(double), h->stream);
  launch_zero(h->d.scal + SC_NFAIL, sizeof(double), h->stream);
  launch_feature_invert(h->d, lambda, kappa_max, h->stream);
  launch_camera_pass_b(h->d, lambda, h->stream);
  check_launch("assemble");
  h->last_lambda = lambda;
}

// block-Jacobi blocks, and the coarse space of the two-level preconditioners: the
// similarity gauge, plus the network's vectors for BA_PC_LEARNED
void assemble_precond(ba_handle* h, double lambda) {
  launch_precond_blockjacobi(h->d, h->stream);
  h->d.coarse_k = 0;
  const bool learned = h->precond == BA_PC_LEARNED && ba_gnn_impl::ready(h->gnn);
  const bool resolved = h->d.fp64 || lambda >= COARSE_MIN_DAMPING_FP32;
  if ((h->precond == BA_PC_GAUGE || learned) && h->d.nA > 0 && resolved && lambda <= COARSE_MAX_DAMPING) {
    launch_gauge_basis(h->d, h->stream);
    h->d.coarse_k = COARSE_GAUGE;
    if (learned) {
      ba_gnn_impl::apply(h->gnn, h->d, lambda, h->stream);
      h->d.coarse_k = COARSE_K;
    }
    launch_coarse_setup(h->d, lambda, h->stream);
  }
  check_launch("preconditioner");
}

void assemble(ba_handle* h, double lambda, double kappa_max) {
  assemble_schur(h, lambda, kappa_max);
  assemble_precond(h, lambda);
}

// returns iterations done; with mv_ms, times every product launch with events
int pcg(ba_handle* h, double lambda, double tol, int maxit, double* mv_ms = nullptr) {
  if (h->d.nA == 0) {
    for (int k = 0; k < SC_COUNT; ++k) h->hscal[k] = 0;
    if (mv_ms) *mv_ms = 0;
    return 0;
  }
  launch_pcg_init(h->d, tol, maxit, h->stream);
  int launched = 0;
  for (;;) {
    for (int k = 0; k < PCG_CHECK_EVERY && launched < maxit; ++k, ++launched) {
      if (mv_ms) {
        while (h->mv_ev.size() < 2 * (size_t)(launched + 1)) {
          hipEvent_t e;
          HIPCHK(hipEventCreate(&e));
          h->mv_ev.push_back(e);
        }
        HIPCHK(hipEventRecord(h->mv_ev[2 * launched], h->stream));
      }
      launch_pcg_product(h->d, h->stream);
      if (mv_ms) HIPCHK(hipEventRecord(h->mv_ev[2 * launched + 1], h->stream));
      launch_pcg_update(h->d, lambda, launched, h->stream);
    }
    check_launch("pcg");
    read_scal(h);
    if (h->hscal[SC_DONE] != 0.0 || launched >= maxit) break;
  }
  const int iters = (int)h->hscal[SC_ITER];
  if (mv_ms) {
    // the products of the iterations that ran (later launches exit at once)
    double t = 0;
    const int real = std::min(launched, iters + (h->hscal[SC_BREAK] != 0.0 ? 1 : 0));
    for (int k = 0; k < real; ++k) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, h->mv_ev[2 * k], h->mv_ev[2 * k + 1]));
      t += ms;
    }
    *mv_ms = t;
  }
  return iters;
}

void record(ba_handle* h, int phase) {
  if (h->events) HIPCHK(hipEventRecord(h->ev[phase], h->stream));
}

ba_status guard(ba_handle* h, const std::function<void()>& fn) {
  try {
    fn();
    return BA_OK;
  } catch (const BaError& e) {
    if (h) h->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (h) h->err = "host allocation failed";
    return BA_E_OOM;
  } catch (const std::exception& e) {
    if (h) h->err = e.what();
    return BA_E_DEVICE;
  }
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// one shape from its 16-double C-ABI record into the device layout (ba_shape.h)
void shape_from_abi(int t, const double* p, double* o) {
  std::fill(o, o + SH_STRIDE, 0.0);
  if (!finite_all(p, 16)) throw BaError(BA_E_INVALID, "non-finite shape parameter");
  auto rotation = [&](const double* R) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double v = R[3 * i] * R[3 * j] + R[3 * i + 1] * R[3 * j + 1] + R[3 * i + 2] * R[3 * j + 2];
        if (std::fabs(v - (i == j ? 1.0 : 0.0)) > 1e-6) throw BaError(BA_E_INVALID, "shape rotation is not orthonormal");
      }
    double c[3];
    cross(R, R + 3, c);
    if (c[0] * R[6] + c[1] * R[7] + c[2] * R[8] < 0) throw BaError(BA_E_INVALID, "shape rotation is a reflection");
    std::copy_n(R, 9, o);
  };
  auto positive = [](double v, const char* what) {
    if (!(v > 0)) throw BaError(BA_E_INVALID, std::string("shape ") + what + " must be positive");
    return std::log(v);
  };
  switch (t) {
    case SH_SPHERE:
      std::copy_n(p, 3, o);
      o[3] = positive(p[3], "radius");
      break;
    case SH_CYLINDER: {
      const double nd = norm3(p);
      if (!(nd > 0)) throw BaError(BA_E_INVALID, "cylinder axis direction is zero");
      const double Q[3] = {p[3] + p[0] / nd, p[4] + p[1] / nd, p[5] + p[2] / nd};
      if (!line_from_points(p + 3, Q, o)) throw BaError(BA_E_INVALID, "bad cylinder axis");
      o[11] = positive(p[6], "radius");
      break;
    }
    case SH_CONE: {
      const double nd = norm3(p + 3);
      if (!(nd > 0)) throw BaError(BA_E_INVALID, "cone axis direction is zero");
      if (!(p[6] < 0.5 * M_PI)) throw BaError(BA_E_INVALID, "cone half-angle must be below pi/2");
      std::copy_n(p, 3, o);
      for (int k = 0; k < 3; ++k) o[3 + k] = p[3 + k] / nd;
      sphere_basis(o + 3, o + 6, o + 9);
      o[12] = positive(p[6], "half-angle");
      break;
    }
    case SH_ELLIPSOID:
      rotation(p);
      std::copy_n(p + 9, 3, o + 9);
      for (int k = 0; k < 3; ++k) o[12 + k] = positive(p[12 + k], "semi-axis");
      break;
    case SH_CUBOID:
      rotation(p);
      std::copy_n(p + 9, 6, o + 9);
      break;
    default:
      throw BaError(BA_E_INVALID, "unknown shape type " + std::to_string(t));
  }
  o[15] = t;
}

// the device layout of one shape back into its C-ABI record
void shape_to_abi(const double* o, double* p) {
  std::fill(p, p + 16, 0.0);
  switch ((int)o[15]) {
    case SH_SPHERE: std::copy_n(o, 3, p); p[3] = std::exp(o[3]); break;
    case SH_CYLINDER:
      for (int k = 0; k < 3; ++k) { p[k] = o[k]; p[3 + k] = o[10] / o[9] * o[6 + k]; }
      p[6] = std::exp(o[11]);
      break;
    case SH_CONE: std::copy_n(o, 6, p); p[6] = std::exp(o[12]); break;
    case SH_ELLIPSOID:
      std::copy_n(o, 12, p);
      for (int k = 0; k < 3; ++k) p[12 + k] = std::exp(o[12 + k]);
      break;
    default: std::copy_n(o, 15, p); break;
  }
}

void fill_params(ba_handle* h, const double* cams, const double* pts, const double* lines, const double* planes,
                 const double* vps) {
  if (cams) {
    if (!finite_all(cams, (size_t)h->nc * 10)) throw BaError(BA_E_INVALID, "non-finite camera parameter");
    h->cam.assign((size_t)h->nc * CAM_STRIDE, 0.0);
    for (int i = 0; i < h->nc; ++i) {
      const double* c = cams + 10 * (size_t)i;
      double* o = &h->cam[(size_t)CAM_STRIDE * i];
      if (!(c[0] * c[0] + c[1] * c[1] + c[2] * c[2] + c[3] * c[3] > 0)) throw BaError(BA_E_INVALID, "zero quaternion");
      quat_to_R(c, o);
      for (int k = 0; k < 3; ++k) o[9 + k] = c[4 + k];
      o[12] = c[7]; o[13] = c[8]; o[14] = c[9];
    }
  }
  if (pts) {
    if (!finite_all(pts, (size_t)h->np * 3)) throw BaError(BA_E_INVALID, "non-finite point");
    h->pt.assign((size_t)h->np * PT_STRIDE, 0.0);
    for (int i = 0; i < h->np; ++i)
      for (int k = 0; k < 3; ++k) h->pt[(size_t)PT_STRIDE * i + k] = pts[3 * (size_t)i + k];
  }
  if (lines) {
    if (!finite_all(lines, (size_t)h->nl * 6)) throw BaError(BA_E_INVALID, "non-finite line");
    h->ln.assign((size_t)h->nl * LN_STRIDE, 0.0);
    for (int i = 0; i < h->nl; ++i)
      if (!line_from_points(lines + 6 * (size_t)i, lines + 6 * (size_t)i + 3, &h->ln[(size_t)LN_STRIDE * i]))
        throw BaError(BA_E_INVALID, "line " + std::to_string(i) + " has coincident points");
  }
  if (planes) {
    if (!finite_all(planes, (size_t)h->ng * 4)) throw BaError(BA_E_INVALID, "non-finite plane");
    h->pl.assign((size_t)h->ng * PL_STRIDE, 0.0);
    for (int i = 0; i < h->ng; ++i) {
      const double* p = planes + 4 * (size_t)i;
      if (std::fabs(norm3(p) - 1.0) > 1e-6) throw BaError(BA_E_INVALID, "plane normal is not unit");
      double* o = &h->pl[(size_t)PL_STRIDE * i];
      for (int k = 0; k < 4; ++k) o[k] = p[k];
      sphere_basis(o, o + 4, o + 7);
    }
  }
  if (vps) {
    if (!finite_all(vps, (size_t)h->nv * 3)) throw BaError(BA_E_INVALID, "non-finite VP");
    h->vp.assign((size_t)h->nv * VP_STRIDE, 0.0);
    for (int i = 0; i < h->nv; ++i) {
      const double* v = vps + 3 * (size_t)i;
      if (std::fabs(norm3(v) - 1.0) > 1e-6) throw BaError(BA_E_INVALID, "VP is not unit");
      double* o = &h->vp[(size_t)VP_STRIDE * i];
      for (int k = 0; k < 3; ++k) o[k] = v[k];
      sphere_basis(o, o + 4, o + 7);
    }
  }
}

// swap current / candidate parameter sets after an accepted step
void accept_candidate(ba_handle* h) {
  Dev& d = h->d;
  std::swap(d.cam64, d.cam64n); std::swap(d.pt64, d.pt64n); std::swap(d.ln64, d.ln64n);
  std::swap(d.pl64, d.pl64n); std::swap(d.vp64, d.vp64n); std::swap(d.sh64, d.sh64n);
}

void current_cost(ba_handle* h) {
  launch_cost(h->d, false, h->stream);
  read_scal(h);
  h->E = h->hscal[SC_E];
  h->Epix = h->hscal[SC_EPIX];
  h->have_cost = true;
}

ba_solve_options opts_or_default(const ba_solve_options* o) {
  ba_solve_options r;
  ba_default_options(&r);
  if (o) r = *o;
  return r;
}

// one LM step; with stop_grad > 0, a fresh linearisation whose |g|_inf is below it ends
// the solve instead (returns false: no step taken, nothing changed but the linearisation)
bool do_step(ba_handle* h, const ba_solve_options& o, ba_step_report* rep, double stop_grad = 0) {
  set_device(h);
  if (!h->finalized) finalize(h);
  h->d.det = o.deterministic ? 1 : 0;
  if (h->d.det && h->ns > 0) throw BaError(BA_E_INVALID, "the deterministic mode does not take surface groups (shapes)");
  if (h->first_step) {
    h->lambda = o.lambda0;
    h->nu = o.nu0;
    h->first_step = false;
  }
  if (!h->have_cost) current_cost(h);
  if (!std::isfinite(h->E)) throw BaError(BA_E_NUMERIC, "initial cost is not finite");
  ba_step_report r;
  std::memset(&r, 0, sizeof(r));
  r.E_before = h->E;
  r.Epix_before = h->Epix;
  r.lambda = h->lambda;
  record(h, 0);
  const bool relin = h->need_lin;
  if (relin) {
    linearize_all(h);
    if (stop_grad > 0) {
      read_scal(h);
      if (h->hscal[SC_GINF] < stop_grad) {
        r.grad_inf = h->hscal[SC_GINF];
        r.n_degenerate = (int)h->hscal[SC_NDEG];
        r.relinearized = 1;
        r.E_after = r.E_before;
        r.Epix_after = r.Epix_before;
        if (rep) *rep = r;
        return false;
      }
    }
  }
  record(h, 1);
  assemble_schur(h, h->lambda, o.kappa_max);
  record(h, 2);
  const bool fixa = o.fix_a_side != 0;
  const bool dense = !fixa && o.linear_solver == BA_SOLVER_DENSE;
  bool solved = true;
  double mv_ms = 0;
  if (fixa) {
    // cameras and groups held fixed: h_a = 0, the features alone (back-substitution)
    record(h, 3);
    if (h->d.nA) launch_zero(h->d.x, (size_t)h->d.nA * sizeof(double), h->stream);
    read_scal(h);
    r.pcg_iters = 0;
    r.coarse = 0;
  } else if (dense) {
    // direct solve: S formed and factored (the preconditioner phase is empty)
    record(h, 3);
    solved = dense_solve(h, h->lambda);
    if (solved) {
      launch_dense_residual(h->d, h->lambda, h->stream);
      check_launch("dense solve residual");
    }
    read_scal(h);
    r.pcg_iters = 0;
    r.coarse = 0;
    if (!solved) r.pcg_flags |= BA_SOLVE_NOT_SPD;
  } else {
    assemble_precond(h, h->lambda);
    record(h, 3);
    r.pcg_iters = pcg(h, h->lambda, o.pcg_tol, o.pcg_max_iters, o.time_kernels ? &mv_ms : nullptr);
    r.coarse = h->d.coarse_k > 0 && h->hscal[SC_COARSE] != 0.0 ? h->d.coarse_k : 0;
  }
  if (!dense && !fixa && h->hscal[SC_BREAK] != 0.0) r.pcg_flags |= BA_PCG_BREAKDOWN;
  if (r.coarse > 0 && (h->hscal[SC_BREAK] != 0.0 || !std::isfinite(h->hscal[SC_RR]) || !std::isfinite(h->hscal[SC_RZ]))) {
    // the two-level solve broke down: solve again with block-Jacobi alone
    h->d.coarse_k = 0;
    r.coarse = 0;
    r.pcg_flags |= BA_PCG_COARSE_FALLBACK;
    double mv2 = 0;
    r.pcg_iters += pcg(h, h->lambda, o.pcg_tol, o.pcg_max_iters, o.time_kernels ? &mv2 : nullptr);
    mv_ms += mv2;
  }
  r.matvec_ms = mv_ms;
  r.matvec_count = o.time_kernels && !dense && !fixa ? r.pcg_iters + (h->hscal[SC_BREAK] != 0.0 ? 1 : 0) : 0;
  record(h, 4);
  const double rr = h->hscal[SC_RR], bb = h->hscal[SC_BB];
  if (solved && !fixa && !std::isfinite(bb)) r.pcg_flags |= BA_PCG_NONFINITE_RHS;
  r.pcg_rel_residual = solved && !fixa && bb > 0 ? std::sqrt(rr / bb) : 0.0;
  r.n_fp64_blocks = (int)h->hscal[SC_NFLAG];
  r.n_fp64_failed = (int)h->hscal[SC_NFAIL];
  r.n_degenerate = (int)h->hscal[SC_NDEG];
  r.grad_inf = h->hscal[SC_GINF];
  double En = NAN, Epn = NAN, dL = 0;
  if (solved) {
    launch_backsub(h->d, h->stream);
    record(h, 5);
    launch_retract(h->d, h->stream);
    launch_cost(h->d, true, h->stream);
    record(h, 6);
    check_launch("backsub / retract / cost");
    read_scal(h);
    En = h->hscal[SC_E];
    Epn = h->hscal[SC_EPIX];
    dL = -h->hscal[SC_GH] - 0.5 * h->hscal[SC_JH2];
  } else {
    // no step: S is not positive definite; rejected like a step without decrease
    record(h, 5);
    record(h, 6);
    sync(h);
  }
  const double rho = dL > 0 ? (h->E - En) / dL : -INFINITY;
  r.E_after = En;
  r.Epix_after = Epn;
  r.model_decrease = dL;
  r.gain_ratio = rho;
  r.relinearized = relin ? 1 : 0;
  if (std::isfinite(En) && rho > 0) {
    accept_candidate(h);
    h->E = En;
    h->Epix = Epn;
    const double t = 2.0 * rho - 1.0;
    h->lambda = std::max(h->lambda * std::max(1.0 / 3.0, 1.0 - t * t * t), 1e-10);
    h->nu = 2.0;
    h->need_lin = true;
    r.accepted = 1;
  } else {
    h->lambda *= h->nu;
    h->nu *= 2.0;
    // a non-finite reduced system is not cured by more damping of the same linearisation
    if (r.pcg_flags & BA_PCG_NONFINITE_RHS) h->need_lin = true;
  }
  if (h->events) {
    float ms = 0;
    const int map[7][2] = {{0, 1}, {1, 1}, {1, 2}, {2, 3}, {3, 4}, {4, 5}, {5, 6}};
    for (int k = 0; k < 7; ++k) {
      ms = 0;
      if (map[k][0] != map[k][1]) HIPCHK(hipEventElapsedTime(&ms, h->ev[map[k][0]], h->ev[map[k][1]]));
      r.ms[k] = ms;
    }
    r.ms[BA_PHASE_FEATURE] = 0;  // accumulation is timed with linearisation
  }
  if (rep) *rep = r;
  return true;
}

void check_index(const int32_t* v, int64_t n, int hi, const char* what) {
  for (int64_t i = 0; i < n; ++i)
    if (v[i] < 0 || v[i] >= hi) throw BaError(BA_E_INVALID, std::string(what) + " index out of range");
}

}  // namespace

// ===========================================================================
// C ABI
extern "C" {

void ba_default_options(ba_solve_options* o) {
  if (!o) return;
  o->max_iters = 100;
  o->func_tol = 1e-6;
  o->grad_tol = 1e-10;
  o->pcg_tol = 1e-6;
  o->pcg_max_iters = 1000;
  o->lambda0 = 1e-4;
  o->nu0 = 2.0;
  o->kappa_max = 1e4;
  o->time_kernels = 0;
  o->deterministic = 0;
  o->linear_solver = BA_SOLVER_PCG;
  o->fix_a_side = 0;
}

void ba_default_reliability_options(ba_reliability_options* o) {
  if (!o) return;
  o->min_active_obs = 3;
  o->max_sigma_point = 0.01;
  o->max_sigma_line = 0.1;
  o->min_group_support = 3;
}

ba_status ba_create(const ba_problem_desc* desc, ba_handle** out) {
  if (!out) return BA_E_INVALID;
  *out = nullptr;
  if (!desc) return BA_E_INVALID;
  ba_handle* h = new (std::nothrow) ba_handle();
  if (!h) return BA_E_OOM;
  ba_status st = guard(h, [&] {
    if (desc->n_cameras < 0 || desc->n_points < 0 || desc->n_lines < 0 || desc->n_planes < 0 || desc->n_vps < 0)
      throw BaError(BA_E_INVALID, "negative count");
    if (desc->camera_dof != 6 && desc->camera_dof != 9) throw BaError(BA_E_INVALID, "camera_dof must be 6 or 9");
    if (desc->precision != BA_PREC_FP64 && desc->precision != BA_PREC_MIXED) throw BaError(BA_E_INVALID, "bad precision");
    if (desc->precond != BA_PC_BLOCK_JACOBI && desc->precond != BA_PC_LEARNED && desc->precond != BA_PC_GAUGE)
      throw BaError(BA_E_INVALID, "bad precond");
    if (!std::isfinite(desc->cx) || !std::isfinite(desc->cy)) throw BaError(BA_E_INVALID, "non-finite principal point");
    h->nc = desc->n_cameras; h->np = desc->n_points; h->nl = desc->n_lines; h->ng = desc->n_planes; h->nv = desc->n_vps;
    h->CD = desc->camera_dof; h->cx = desc->cx; h->cy = desc->cy;
    h->precision = desc->precision; h->precond = desc->precond; h->device = desc->device;
    if ((h->nc && !desc->cameras) || (h->np && !desc->points) || (h->nl && !desc->lines) || (h->ng && !desc->planes) ||
        (h->nv && !desc->vps))
      throw BaError(BA_E_INVALID, "missing parameter array");
    fill_params(h, desc->cameras, desc->points, desc->lines, desc->planes, desc->vps);
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (h->device < 0 || h->device >= ndev) throw BaError(BA_E_INVALID, "bad device index");
    set_device(h);
    noalloc_scratch(h->device);
    if (desc->hip_stream) {
      h->stream = (hipStream_t)desc->hip_stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
      h->own_stream = true;
    }
    for (int k = 0; k <= BA_PHASE_COUNT; ++k) HIPCHK(hipEventCreate(&h->ev[k]));
    h->events = true;
    for (int k = 0; k < 13; ++k) h->obs[k].loss = default_loss(k);
  });
  if (st != BA_OK) {
    ba_destroy(h);
    return st;
  }
  *out = h;
  return BA_OK;
}

ba_status ba_add_observations(ba_handle* h, int32_t kind, int64_t n, const int32_t* a, const int32_t* b,
                              const double* meas, const ba_loss* loss) {
  if (!h) return BA_E_INVALID;
  return guard(h, [&] {
    if (h->finalized) throw BaError(BA_E_STATE, "observations must be added before the first step");
    if (kind < 0 || kind > 12) throw BaError(BA_E_INVALID, "bad kind");
    if (n < 0 || (n > 0 && (!a || !b))) throw BaError(BA_E_INVALID, "bad arrays");
    const bool has_meas = kind == BA_OBS_POINT || kind == BA_OBS_LINE;
    if (has_meas && n > 0 && !meas) throw BaError(BA_E_INVALID, "measurements required");
    int ha = 0, hb = 0;
    switch (kind) {
      case BA_OBS_POINT: ha = h->nc; hb = h->np; break;
      case BA_OBS_LINE: ha = h->nc; hb = h->nl; break;
      case BA_ASSOC_PLANE_POINT: ha = h->ng; hb = h->np; break;
      case BA_ASSOC_PLANE_LINE: ha = h->ng; hb = h->nl; break;
      case BA_ASSOC_VP_LINE: ha = h->nv; hb = h->nl; break;
      case BA_ASSOC_JUNCTION: ha = h->np; hb = h->nl; break;
      case BA_REL_VP_ORTHO: case BA_REL_VP_PARALLEL: ha = hb = h->nv; break;
      case BA_ASSOC_PLANE_POINT_3D: ha = h->ng; hb = h->np; break;
      case BA_REL_PLANE_ORTHO: case BA_REL_PLANE_PARALLEL: ha = hb = h->ng; break;
      case BA_ASSOC_SHAPE_POINT: ha = h->ns; hb = h->np; break;
      case BA_ASSOC_SHAPE_LINE: ha = h->ns; hb = h->nl; break;
    }
    check_index(a, n, ha, "first");
    check_index(b, n, hb, "second");
    if (kind >= BA_REL_VP_ORTHO && kind <= BA_REL_PLANE_PARALLEL)
      for (int64_t i = 0; i < n; ++i)
        if (a[i] == b[i]) throw BaError(BA_E_INVALID, "a relation needs two distinct groups");
    if (has_meas && !finite_all(meas, (size_t)n * 4)) throw BaError(BA_E_INVALID, "non-finite measurement");
    if (loss) {
      if (loss->kind < 0 || loss->kind > 2 || !(loss->scale > 0) || !(loss->weight > 0) || !std::isfinite(loss->scale) ||
          !std::isfinite(loss->weight))
        throw BaError(BA_E_INVALID, "bad loss");
      h->obs[kind].loss = *loss;
      h->obs[kind].loss_set = true;
    }
    Obs& o = h->obs[kind];
    o.a.insert(o.a.end(), a, a + n);
    o.b.insert(o.b.end(), b, b + n);
    if (has_meas) o.meas.insert(o.meas.end(), meas, meas + 4 * n);
  });
}

ba_status ba_add_shapes(ba_handle* h, int64_t n, const int32_t* types, const double* params) {
  if (!h) return BA_E_INVALID;
  return guard(h, [&] {
    if (h->finalized) throw BaError(BA_E_STATE, "shapes must be added before the first step");
    if (n < 0 || (n > 0 && (!types || !params))) throw BaError(BA_E_INVALID, "bad arrays");
    if ((int64_t)h->ns + n > INT32_MAX / SH_DOF) throw BaError(BA_E_INVALID, "too many shapes");
    std::vector<double> add((size_t)n * SH_STRIDE);
    for (int64_t i = 0; i < n; ++i) shape_from_abi(types[i], params + 16 * i, &add[(size_t)SH_STRIDE * i]);
    h->sh.insert(h->sh.end(), add.begin(), add.end());
    h->ns += (int)n;
  });
}

ba_status ba_get_shapes(const ba_handle* hc, double* params) {
  ba_handle* h = const_cast<ba_handle*>(hc);
  if (!h) return BA_E_INVALID;
  return guard(h, [&] {
    std::vector<double> sh = h->sh;
    if (h->finalized && !sh.empty()) {
      set_device(h);
      HIPCHK(hipMemcpyAsync(sh.data(), h->d.sh64, sh.size() * 8, hipMemcpyDeviceToHost, h->stream));
      sync(h);
    }
    if (params)
      for (int i = 0; i < h->ns; ++i) shape_to_abi(&sh[(size_t)SH_STRIDE * i], params + 16 * (size_t)i);
  });
}

ba_status ba_lm_step(ba_handle* h, const ba_solve_options* opt, ba_step_report* rep) {
  if (!h) return BA_E_INVALID;
  const ba_solve_options o = opts_or_default(opt);
  return guard(h, [&] { do_step(h, o, rep); });
}

namespace {
// LM to termination (see ba_solve)
void solve_loop(ba_handle* h, const ba_solve_options& o, ba_summary& s) {
  std::memset(&s, 0, sizeof(s));
  s.termination = 2;
  auto t0 = std::chrono::steady_clock::now();
  set_device(h);
  if (!h->finalized) finalize(h);
  if (!h->have_cost) current_cost(h);
  s.E_initial = h->E;
  for (int it = 0; it < o.max_iters; ++it) {
    ba_step_report r;
    if (!do_step(h, o, &r, o.grad_tol)) { s.termination = 1; break; }
    s.iters++;
    s.pcg_iters_total += r.pcg_iters;
    if (r.accepted) {
      s.accepted++;
      const double rel = std::fabs(r.Epix_before - r.Epix_after) / std::max(r.Epix_before, 1e-300);
      if (rel < o.func_tol) { s.termination = 0; break; }
    }
    if (h->lambda > 1e16) { s.termination = 3; break; }
  }
  s.E_final = h->E;
  s.Epix_final = h->Epix;
  s.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// record mask in internal order (empty vector: nothing left out of that kind)
void apply_mask(ba_handle* h, const std::vector<uint8_t>& pt, const std::vector<uint8_t>& ln,
                const std::vector<uint8_t>& pl, const std::vector<uint8_t>& vp) {
  Dev& d = h->d;
  auto put = [&](uint8_t* dst, const std::vector<uint8_t>& v, int n) {
    if (!n) return false;
    if (v.empty()) {
      launch_zero(dst, n, h->stream);
      return false;
    }
    HIPCHK(hipMemcpyAsync(dst, v.data(), n, hipMemcpyHostToDevice, h->stream));
    return std::any_of(v.begin(), v.end(), [](uint8_t x) { return x != 0; });
  };
  bool any = false;
  any |= put(d.mpt, pt, h->np);
  any |= put(d.mln, ln, h->nl);
  any |= put(d.mpl, pl, h->ng);
  any |= put(d.mvp, vp, h->nv);
  sync(h);
  d.has_mask = any ? 1 : 0;
  h->need_lin = true;
  h->have_cost = false;
}

// per-feature statistics (internal order)
void feature_stats(ba_handle* h, std::vector<int32_t> (&act)[2], std::vector<int32_t> (&obs)[2],
                   std::vector<double> (&sig)[2]) {
  linearize_all(h);
  const int n[2] = {h->np, h->nl};
  DevAlloc tmp;
  struct Release {
    DevAlloc& a;
    ~Release() { a.free_all(); }
  } release{tmp};
  for (int k = 0; k < 2; ++k) {
    act[k].assign(n[k], 0); obs[k].assign(n[k], 0); sig[k].assign(n[k], 0.0);
    if (!n[k]) continue;
    int32_t* da = tmp.get<int32_t>(n[k]);
    int32_t* dn = tmp.get<int32_t>(n[k]);
    double* ds = tmp.get<double>(n[k]);
    launch_feature_stats(h->d, da, dn, ds, k == 0 ? 3 : 4, h->stream);
    check_launch("feature statistics");
    HIPCHK(hipMemcpyAsync(act[k].data(), da, n[k] * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(obs[k].data(), dn, n[k] * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(sig[k].data(), ds, n[k] * 8, hipMemcpyDeviceToHost, h->stream));
    sync(h);
  }
}
}  // namespace

ba_status ba_solve(ba_handle* h, const ba_solve_options* opt, ba_summary* sum) {
  if (!h) return BA_E_INVALID;
  const ba_solve_options o = opts_or_default(opt);
  ba_summary s;
  std::memset(&s, 0, sizeof(s));
  s.termination = 2;
  ba_status st = guard(h, [&] { solve_loop(h, o, s); });
  if (sum) *sum = s;
  if (st != BA_OK) return st;
  return s.termination == 2 ? BA_E_NOT_CONVERGED : BA_OK;
}

ba_status ba_set_record_mask(ba_handle* h, const uint8_t* points_out, const uint8_t* lines_out,
                             const uint8_t* planes_out, const uint8_t* vps_out) {
  if (!h) return BA_E_INVALID;
  return guard(h, [&] {
    set_device(h);
    if (!h->finalized) finalize(h);
    std::vector<uint8_t> pt, ln, pl, vp;
    if (points_out) {
      pt.assign(h->np, 0);
      for (int j = 0; j < h->np; ++j) pt[h->pt_inv[j]] = points_out[j] ? 1 : 0;
    }
    if (lines_out) {
      ln.assign(h->nl, 0);
      for (int k = 0; k < h->nl; ++k) ln[h->ln_inv[k]] = lines_out[k] ? 1 : 0;
    }
    if (planes_out) pl.assign(planes_out, planes_out + h->ng);
    if (vps_out) vp.assign(vps_out, vps_out + h->nv);
    apply_mask(h, pt, ln, pl, vp);
  });
}

ba_status ba_feature_reliability(ba_handle* h, int32_t* pt_active, int32_t* pt_obs, double* pt_sigma,
                                 int32_t* ln_active, int32_t* ln_obs, double* ln_sigma) {
  if (!h) return BA_E_INVALID;
  return guard(h, [&] {
    set_device(h);
    if (!h->finalized) finalize(h);
    std::vector<int32_t> act[2], obs[2];
    std::vector<double> sig[2];
    feature_stats(h, act, obs, sig);
    for (int j = 0; j < h->np; ++j) {
      const int i = h->pt_inv[j];
      if (pt_active) pt_active[j] = act[0][i];
      if (pt_obs) pt_obs[j] = obs[0][i];
      if (pt_sigma) pt_sigma[j] = sig[0][i];
    }
    for (int k = 0; k < h->nl; ++k) {
      const int i = h->ln_inv[k];
      if (ln_active) ln_active[k] = act[1][i];
      if (ln_obs) ln_obs[k] = obs[1][i];
      if (ln_sigma) ln_sigma[k] = sig[1][i];
    }
  });
}

ba_status ba_solve_two_stage(ba_handle* h, const ba_solve_options* opt, const ba_reliability_options* ro,
                             ba_two_stage_summary* out) {
  if (!h) return BA_E_INVALID;
  ba_solve_options o = opts_or_default(opt);
  ba_reliability_options r;
  ba_default_reliability_options(&r);
  if (ro) r = *ro;
  ba_two_stage_summary sum;
  std::memset(&sum, 0, sizeof(sum));
  const ba_status st = guard(h, [&] {
    if (r.min_active_obs < 0 || !(r.max_sigma_point >= 0) || !(r.max_sigma_line >= 0) || r.min_group_support < 0)
      throw BaError(BA_E_INVALID, "bad reliability options");
    set_device(h);
    if (!h->finalized) finalize(h);
    const std::vector<uint8_t> none;
    apply_mask(h, none, none, none, none);
    std::vector<int32_t> act[2], obs[2];
    std::vector<double> sig[2];
    feature_stats(h, act, obs, sig);
    // reliable flags (internal order)
    std::vector<uint8_t> rel[2];
    for (int k = 0; k < 2; ++k) {
      const double smax = k == 0 ? r.max_sigma_point : r.max_sigma_line;
      rel[k].resize(act[k].size());
      for (size_t i = 0; i < act[k].size(); ++i) rel[k][i] = act[k][i] >= r.min_active_obs && sig[k][i] <= smax;
    }
    // group support: distinct reliable features associated with each plane / VP
    auto support = [&](int ngrp, std::initializer_list<std::pair<int, int>> kinds) {
      std::vector<int> cnt(ngrp, 0);
      for (auto [kind, fk] : kinds) {
        const Obs& ob = h->obs[kind];
        std::vector<std::pair<int, int>> pairs;
        for (size_t i = 0; i < ob.a.size(); ++i) pairs.emplace_back(ob.a[i], ob.b[i]);
        std::sort(pairs.begin(), pairs.end());
        pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
        for (auto [g, f] : pairs) {
          const int fi = fk == 0 ? h->pt_inv[f] : h->ln_inv[f];
          if (rel[fk][fi]) cnt[g]++;
        }
      }
      return cnt;
    };
    const std::vector<int> spl = support(h->ng, {{BA_ASSOC_PLANE_POINT, 0}, {BA_ASSOC_PLANE_LINE, 1}});
    const std::vector<int> svp = support(h->nv, {{BA_ASSOC_VP_LINE, 1}});
    std::vector<uint8_t> m1[2], mpl(h->ng), mvp(h->nv), m2[2];
    for (int k = 0; k < 2; ++k) {
      m1[k].resize(rel[k].size());
      m2[k].resize(rel[k].size());
      for (size_t i = 0; i < rel[k].size(); ++i) {
        m1[k][i] = !rel[k][i];
        m2[k][i] = rel[k][i];
      }
    }
    for (int g = 0; g < h->ng; ++g) mpl[g] = spl[g] < r.min_group_support;
    for (int v = 0; v < h->nv; ++v) mvp[v] = svp[v] < r.min_group_support;
    sum.n_points_unreliable = (int)std::count(m1[0].begin(), m1[0].end(), 1);
    sum.n_lines_unreliable = (int)std::count(m1[1].begin(), m1[1].end(), 1);
    sum.n_planes_out = (int)std::count(mpl.begin(), mpl.end(), 1);
    sum.n_vps_out = (int)std::count(mvp.begin(), mvp.end(), 1);
    // stage 1: cameras, reliable features, supported groups
    o.fix_a_side = 0;
    apply_mask(h, m1[0], m1[1], mpl, mvp);
    h->first_step = true;
    solve_loop(h, o, sum.stage1);
    // stage 2: the unreliable features with cameras and groups fixed
    o.fix_a_side = 1;
    apply_mask(h, m2[0], m2[1], none, none);
    h->first_step = true;
    solve_loop(h, o, sum.stage2);
    apply_mask(h, none, none, none, none);
    h->first_step = true;
  });
  if (out) *out = sum;
  return st;
}

ba_status ba_get_parameters(const ba_handle* hc, double* cams, double* pts, double* lines, double* planes, double* vps) {
  ba_handle* h = const_cast<ba_handle*>(hc);
  if (!h) return BA_E_INVALID;
  return guard(h, [&] {
    std::vector<double> cam = h->cam, pt = h->pt, ln = h->ln, pl = h->pl, vp = h->vp;
    if (h->finalized) {
      set_device(h);
      const Dev& d = h->d;
      std::vector<double> ptI(pt.size()), lnI(ln.size());
      if (!cam.empty()) HIPCHK(hipMemcpyAsync(cam.data(), d.cam64, cam.size() * 8, hipMemcpyDeviceToHost, h->stream));
      if (!ptI.empty()) HIPCHK(hipMemcpyAsync(ptI.data(), d.pt64, ptI.size() * 8, hipMemcpyDeviceToHost, h->stream));
      if (!lnI.empty()) HIPCHK(hipMemcpyAsync(lnI.data(), d.ln64, lnI.size() * 8, hipMemcpyDeviceToHost, h->stream));
      if (!pl.empty()) HIPCHK(hipMemcpyAsync(pl.data(), d.pl64, pl.size() * 8, hipMemcpyDeviceToHost, h->stream));
      if (!vp.empty()) HIPCHK(hipMemcpyAsync(vp.data(), d.vp64, vp.size() * 8, hipMemcpyDeviceToHost, h->stream));
      sync(h);
      for (int i = 0; i < h->np; ++i) std::copy_n(&ptI[(size_t)PT_STRIDE * i], PT_STRIDE, &pt[(size_t)PT_STRIDE * h->pt_perm[i]]);
      for (int i = 0; i < h->nl; ++i) std::copy_n(&lnI[(size_t)LN_STRIDE * i], LN_STRIDE, &ln[(size_t)LN_STRIDE * h->ln_perm[i]]);
    }
    if (cams)
      for (int i = 0; i < h->nc; ++i) {
        const double* c = &cam[(size_t)CAM_STRIDE * i];
        double* o = cams + 10 * (size_t)i;
        R_to_quat(c, o);
        for (int k = 0; k < 3; ++k) o[4 + k] = c[9 + k];
        o[7] = c[12]; o[8] = c[13]; o[9] = c[14];
      }
    if (pts)
      for (int i = 0; i < h->np; ++i)
        for (int k = 0; k < 3; ++k) pts[3 * (size_t)i + k] = pt[(size_t)PT_STRIDE * i + k];
    if (lines)
      for (int i = 0; i < h->nl; ++i) {
        const double* L = &ln[(size_t)LN_STRIDE * i];
        // d = w1 u1 has norm w1; output unit d and m / |d| = (w2 / w1) u2
        for (int k = 0; k < 3; ++k) {
          lines[6 * (size_t)i + k] = L[k];
          lines[6 * (size_t)i + 3 + k] = L[10] / L[9] * L[3 + k];
        }
      }
    if (planes)
      for (int i = 0; i < h->ng; ++i)
        for (int k = 0; k < 4; ++k) planes[4 * (size_t)i + k] = pl[(size_t)PL_STRIDE * i + k];
    if (vps)
      for (int i = 0; i < h->nv; ++i)
        for (int k = 0; k < 3; ++k) vps[3 * (size_t)i + k] = vp[(size_t)VP_STRIDE * i + k];
  });
}

ba_status ba_set_parameters(ba_handle* h, const double* cams, const double* pts, const double* lines,
                            const double* planes, const double* vps) {
  if (!h) return BA_E_INVALID;
  return guard(h, [&] {
    fill_params(h, cams, pts, lines, planes, vps);
    if (h->finalized) {
      set_device(h);
      Dev& d = h->d;
      std::vector<double> ptI((size_t)h->np * PT_STRIDE), lnI((size_t)h->nl * LN_STRIDE);
      for (int i = 0; i < h->np; ++i) std::copy_n(&h->pt[(size_t)PT_STRIDE * h->pt_perm[i]], PT_STRIDE, &ptI[(size_t)PT_STRIDE * i]);
      for (int i = 0; i < h->nl; ++i) std::copy_n(&h->ln[(size_t)LN_STRIDE * h->ln_perm[i]], LN_STRIDE, &lnI[(size_t)LN_STRIDE * i]);
      if (cams) upload(h, d.cam64, h->cam);
      if (pts) upload(h, d.pt64, ptI);
      if (lines) upload(h, d.ln64, lnI);
      if (planes) upload(h, d.pl64, h->pl);
      if (vps) upload(h, d.vp64, h->vp);
      sync(h);
    }
    h->need_lin = true;
    h->have_cost = false;
  });
}

ba_status ba_get_lm_state(const ba_handle* h, double* lambda, double* nu) {
  if (!h) return BA_E_INVALID;
  if (lambda) *lambda = h->lambda;
  if (nu) *nu = h->nu;
  return BA_OK;
}

ba_status ba_set_lm_state(ba_handle* h, double lambda, double nu) {
  if (!h) return BA_E_INVALID;
  if (!(lambda > 0) || !(nu > 1) || !std::isfinite(lambda) || !std::isfinite(nu)) {
    h->err = "lambda must be > 0 and nu > 1";
    return BA_E_INVALID;
  }
  h->lambda = lambda;
  h->nu = nu;
  h->first_step = false;
  return BA_OK;
}

ba_status ba_linearize(ba_handle* h, double lambda) {
  if (!h) return BA_E_INVALID;
  return guard(h, [&] {
    if (!(lambda >= 0) || !std::isfinite(lambda)) throw BaError(BA_E_INVALID, "bad lambda");
    set_device(h);
    if (!h->finalized) finalize(h);
    linearize_all(h);
    ba_solve_options o;
    ba_default_options(&o);
    assemble(h, lambda, o.kappa_max);
    sync(h);
  });
}

ba_status ba_record_count(const ba_handle* h, int32_t family, int64_t* count) {
  if (!h || family < 1 || family > 14 || !count) return BA_E_INVALID;
  if (!h->finalized) { const_cast<ba_handle*>(h)->err = "records exist after the first step"; return BA_E_STATE; }
  if (family >= 8 && family <= 11) *count = std::count(h->rel_kind.begin(), h->rel_kind.end(), family - 8);
  else *count = h->d.fn[family >= 12 ? family - 4 : family];
  return BA_OK;
}

namespace {
// relation family 8..11: the records of kind family - 8
ba_status export_relations(ba_handle* h, int32_t fam, int64_t* keys, double* r, double* J) {
  return guard(h, [&] {
    if (!h->finalized) throw BaError(BA_E_STATE, "no records yet");
    const int kind = fam - 8, rows = (kind == 1 || kind == 3) ? 3 : 1, gd = kind >= 2 ? 3 : 2;
    const int n = h->d.n_rel;
    std::vector<double> rr(3 * (size_t)n), JJ(18 * (size_t)n);
    if ((r || J) && n) {
      set_device(h);
      HIPCHK(hipMemcpyAsync(rr.data(), h->d.rel_r, rr.size() * 8, hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipMemcpyAsync(JJ.data(), h->d.rel_J, JJ.size() * 8, hipMemcpyDeviceToHost, h->stream));
      sync(h);
    }
    int64_t o = 0;
    for (int i = 0; i < n; ++i) {
      if (h->rel_kind[i] != kind) continue;
      if (keys) { keys[3 * o] = -1; keys[3 * o + 1] = h->rel_ga[i]; keys[3 * o + 2] = h->rel_gb[i]; }
      for (int row = 0; row < rows; ++row) {
        if (r) r[o * rows + row] = rr[3 * (size_t)i + row];
        if (J)
          for (int side = 0; side < 2; ++side)
            for (int c = 0; c < gd; ++c)
              J[(o * rows + row) * 2 * gd + side * gd + c] = JJ[((size_t)i * 3 + row) * 6 + 3 * side + c];
      }
      ++o;
    }
  });
}
}  // namespace

ba_status ba_export_records(const ba_handle* hc, int32_t fam, int64_t* keys, double* r, double* J) {
  ba_handle* h = const_cast<ba_handle*>(hc);
  if (!h || fam < 1 || fam > 14) return BA_E_INVALID;
  if (fam >= 8 && fam <= 11) return export_relations(h, fam, keys, r, J);
  if (fam >= 12) fam -= 4;  // 3D point-to-plane, shape point, shape line: stored as 8, 9, 10
  return guard(h, [&] {
    if (!h->finalized) throw BaError(BA_E_STATE, "no records yet");
    const int64_t n = h->d.fn[fam];
    if (keys) std::copy(h->keys[fam].begin(), h->keys[fam].end(), keys);
    if (!r && !J) return;
    const int stride = slot_stride(fam, h->CD), rows = fam_rows(fam);
    const int nc = slot_nc(fam, h->CD), ng = slot_ng(fam), nf = slot_nf(fam);
    const int ncol = (fam == 5 || fam == 8 ? 0 : h->CD) + nf + ng;
    set_device(h);
    auto fetch = [&](const void* src, size_t cnt) {
      std::vector<double> out(cnt);
      if (!cnt) return out;
      if (h->d.fp64) {
        HIPCHK(hipMemcpyAsync(out.data(), src, cnt * 8, hipMemcpyDeviceToHost, h->stream));
        sync(h);
      } else {
        std::vector<float> fb(cnt);
        HIPCHK(hipMemcpyAsync(fb.data(), src, cnt * 4, hipMemcpyDeviceToHost, h->stream));
        sync(h);
        std::copy(fb.begin(), fb.end(), out.begin());
      }
      return out;
    };
    const std::vector<double> buf = fetch(h->d.frec[fam], (size_t)n * stride);
    const std::vector<double> res = fetch(h->d.fres[fam], (size_t)n * rows);
    const int OC = 0, OG = OC + rows * nc, OF = OG + rows * ng;
    for (int64_t i = 0; i < n; ++i) {
      const double* s = &buf[(size_t)i * stride];
      for (int row = 0; row < rows; ++row) {
        if (r) r[(size_t)i * rows + row] = res[(size_t)i * rows + row];
        if (J) {
          double* o = J + ((size_t)i * rows + row) * ncol;
          int col = 0;
          if (fam != 5 && fam != 8) {
            for (int k = 0; k < h->CD; ++k) o[col++] = k < nc ? s[OC + row * nc + k] : 0.0;
          }
          for (int k = 0; k < nf; ++k) o[col++] = s[OF + row * nf + k];
          for (int k = 0; k < ng; ++k) o[col++] = s[OG + row * ng + k];
        }
      }
    }
  });
}

ba_status ba_export_feature_blocks(const ba_handle* hc, double* Vp, double* gp, double* Vl, double* gl) {
  ba_handle* h = const_cast<ba_handle*>(hc);
  if (!h) return BA_E_INVALID;
  return guard(h, [&] {
    if (!h->finalized) throw BaError(BA_E_STATE, "no linearisation yet");
    set_device(h);
    auto fetch = [&](const void* src, size_t n) {
      std::vector<double> out(n);
      if (!n) return out;
      if (h->d.fp64) HIPCHK(hipMemcpyAsync(out.data(), src, n * 8, hipMemcpyDeviceToHost, h->stream));
      else {
        std::vector<float> f(n);
        HIPCHK(hipMemcpyAsync(f.data(), src, n * 4, hipMemcpyDeviceToHost, h->stream));
        sync(h);
        std::copy(f.begin(), f.end(), out.begin());
      }
      sync(h);
      return out;
    };
    auto unpack = [](const double* s, int N, double* o) {
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
          const int a = std::min(i, j), b = std::max(i, j);
          o[i * N + j] = s[a * N - a * (a - 1) / 2 + (b - a)];
        }
    };
    if (Vp || gp) {
      auto V = fetch(h->d.Vp, (size_t)h->np * 6), g = fetch(h->d.gp, (size_t)h->np * 3);
      for (int i = 0; i < h->np; ++i) {
        const int o = h->pt_perm[i];
        if (Vp) unpack(&V[6 * (size_t)i], 3, Vp + 9 * (size_t)o);
        if (gp) for (int k = 0; k < 3; ++k) gp[3 * (size_t)o + k] = g[3 * (size_t)i + k];
      }
    }
    if (Vl || gl) {
      auto V = fetch(h->d.Vl, (size_t)h->nl * 10), g = fetch(h->d.gl, (size_t)h->nl * 4);
      for (int i = 0; i < h->nl; ++i) {
        const int o = h->ln_perm[i];
        if (Vl) unpack(&V[10 * (size_t)i], 4, Vl + 16 * (size_t)o);
        if (gl) for (int k = 0; k < 4; ++k) gl[4 * (size_t)o + k] = g[4 * (size_t)i + k];
      }
    }
  });
}

ba_status ba_export_reduced(const ba_handle* hc, double* b, double* Sc, double* Sp, double* Sv) {
  ba_handle* h = const_cast<ba_handle*>(hc);
  if (!h) return BA_E_INVALID;
  return guard(h, [&] {
    if (!h->finalized) throw BaError(BA_E_STATE, "no linearisation yet");
    set_device(h);
    const Dev& d = h->d;
    if (b && d.nA) HIPCHK(hipMemcpyAsync(b, d.bA, d.nA * 8, hipMemcpyDeviceToHost, h->stream));
    if (Sc && d.nc) HIPCHK(hipMemcpyAsync(Sc, d.Scam, (size_t)d.nc * d.CD * d.CD * 8, hipMemcpyDeviceToHost, h->stream));
    if (Sp && d.ng) HIPCHK(hipMemcpyAsync(Sp, d.Spl, (size_t)d.ng * 9 * 8, hipMemcpyDeviceToHost, h->stream));
    if (Sv && d.nv) HIPCHK(hipMemcpyAsync(Sv, d.Svp, (size_t)d.nv * 4 * 8, hipMemcpyDeviceToHost, h->stream));
    sync(h);
  });
}

ba_status ba_export_shape_blocks(const ba_handle* hc, double* S) {
  ba_handle* h = const_cast<ba_handle*>(hc);
  if (!h) return BA_E_INVALID;
  return guard(h, [&] {
    if (!h->finalized) throw BaError(BA_E_STATE, "no linearisation yet");
    set_device(h);
    if (S && h->ns)
      HIPCHK(hipMemcpyAsync(S, h->d.Ssh, (size_t)h->ns * SH_DOF * SH_DOF * 8, hipMemcpyDeviceToHost, h->stream));
    sync(h);
  });
}

ba_status ba_schur_matvec(ba_handle* h, const double* x, double* y) {
  if (!h || !x || !y) return BA_E_INVALID;
  return guard(h, [&] {
    if (!h->finalized) throw BaError(BA_E_STATE, "no linearisation yet");
    set_device(h);
    const Dev& d = h->d;
    HIPCHK(hipMemcpyAsync(d.z, x, d.nA * 8, hipMemcpyHostToDevice, h->stream));
    launch_schur_matvec(d, d.z, d.q, h->last_lambda, h->stream);
    HIPCHK(hipMemcpyAsync(y, d.q, d.nA * 8, hipMemcpyDeviceToHost, h->stream));
    sync(h);
  });
}

ba_status ba_pcg_solve(ba_handle* h, double tol, int32_t max_iters, double* x, int32_t* iters, double* rel_res) {
  if (!h) return BA_E_INVALID;
  return guard(h, [&] {
    if (!h->finalized) throw BaError(BA_E_STATE, "no linearisation yet");
    set_device(h);
    int it = pcg(h, h->last_lambda, tol, max_iters);
    if (h->d.coarse_k > 0 && h->hscal[SC_COARSE] != 0.0 &&
        (h->hscal[SC_BREAK] != 0.0 || !std::isfinite(h->hscal[SC_RR]) || !std::isfinite(h->hscal[SC_RZ]))) {
      // as in ba_lm_step: a two-level solve that broke down is repeated with block-Jacobi
      const int k = h->d.coarse_k;
      h->d.coarse_k = 0;
      it += pcg(h, h->last_lambda, tol, max_iters);
      h->d.coarse_k = k;
    }
    if (x) HIPCHK(hipMemcpyAsync(x, h->d.x, h->d.nA * 8, hipMemcpyDeviceToHost, h->stream));
    sync(h);
    if (iters) *iters = it;
    if (rel_res) *rel_res = h->hscal[SC_BB] > 0 ? std::sqrt(h->hscal[SC_RR] / h->hscal[SC_BB]) : 0.0;
  });
}

ba_status ba_reduced_dim(const ba_handle* h, int64_t* nA, int32_t* cd) {
  if (!h) return BA_E_INVALID;
  if (nA) *nA = (int64_t)h->CD * h->nc + 3 * h->ng + 2 * h->nv + (int64_t)SH_DOF * h->ns;
  if (cd) *cd = h->CD;
  return BA_OK;
}

ba_status ba_set_gnn_weights(ba_handle* h, const void* blob, size_t bytes) {
  if (!h || !blob) return BA_E_INVALID;
  return guard(h, [&] {
    set_device(h);
    if (!h->gnn) {
      std::string e;
      h->gnn = ba_gnn_impl::create(h->CD, 1, h->device, e);
      if (!h->gnn) throw BaError(BA_E_DEVICE, e);
    }
    std::string e;
    if (!ba_gnn_impl::load(h->gnn, blob, bytes, e)) throw BaError(BA_E_INVALID, e);
    if (h->finalized) ba_gnn_impl::attach(h->gnn, h->graph);
  });
}

ba_status ba_export_gnn_graph(ba_handle* h, int32_t* n_nodes, int32_t* n_edges, float* node_x, int32_t* node_type,
                              int32_t* node_off, float* node_unit, int32_t* edge_src, int32_t* edge_dst,
                              int32_t* edge_rev, float* edge_x) {
  if (!h) return BA_E_INVALID;
  return guard(h, [&] {
    if (!h->finalized) throw BaError(BA_E_STATE, "no linearisation yet");
    const auto& G = h->graph;
    if (!G.valid) throw BaError(BA_E_STATE, "the block graph is built for 1 to " +
                                std::to_string(ba_gnn_impl::MAX_GRAPH_NODES) + " camera / plane / VP blocks");
    if (n_nodes) *n_nodes = G.n_nodes;
    if (n_edges) *n_edges = G.n_edges;
    set_device(h);
    if (node_x) {
      ba_gnn_impl::launch_node_features(h->d, h->g_stat, h->g_type, G.n_nodes, h->last_lambda, G.scale, h->g_x,
                                        h->stream);
      check_launch("node features");
      HIPCHK(hipMemcpyAsync(node_x, h->g_x, G.node_static.size() * 4, hipMemcpyDeviceToHost, h->stream));
      sync(h);
    }
    if (node_type) std::copy(G.node_type.begin(), G.node_type.end(), node_type);
    if (node_off) std::copy(G.node_off.begin(), G.node_off.end(), node_off);
    if (node_unit)
      for (int i = 0; i < G.n_nodes; ++i) {
        float* u = node_unit + 9 * (size_t)i;
        for (int k = 0; k < 9; ++k) u[k] = 0.0f;
        const int t = G.node_type[i];
        for (int k = 0; k < G.node_size[i]; ++k)
          u[k] = (float)((t == 0 && k >= 3 && k < 6) || (t == 1 && k == 2) ? G.scale : 1.0);
      }
    if (edge_src) std::copy(G.edge_src.begin(), G.edge_src.end(), edge_src);
    if (edge_dst) std::copy(G.edge_dst.begin(), G.edge_dst.end(), edge_dst);
    if (edge_rev) std::copy(G.edge_rev.begin(), G.edge_rev.end(), edge_rev);
    if (edge_x) std::copy(G.edge_x.begin(), G.edge_x.end(), edge_x);
  });
}

ba_status ba_export_coarse_space(ba_handle* h, int32_t* k, double* Z, double* SZ) {
  if (!h) return BA_E_INVALID;
  return guard(h, [&] {
    if (!h->finalized) throw BaError(BA_E_STATE, "no linearisation yet");
    set_device(h);
    const Dev& d = h->d;
    const int K = d.coarse_k;
    if (k) *k = K;
    if (K == 0 || (!Z && !SZ)) return;
    std::vector<double> col((size_t)K * d.nA);
    for (int pass = 0; pass < 2; ++pass) {
      double* out = pass == 0 ? Z : SZ;
      if (!out) continue;
      HIPCHK(hipMemcpyAsync(col.data(), pass == 0 ? d.Zc : d.SZc, col.size() * sizeof(double), hipMemcpyDeviceToHost,
                            h->stream));
      sync(h);
      for (int e = 0; e < d.nA; ++e)
        for (int c = 0; c < K; ++c) out[(size_t)e * K + c] = col[(size_t)c * d.nA + e];
    }
  });
}

ba_status ba_export_gauge_basis(ba_handle* h, double* G) {
  if (!h || !G) return BA_E_INVALID;
  return guard(h, [&] {
    if (!h->finalized) throw BaError(BA_E_STATE, "no linearisation yet");
    set_device(h);
    const Dev& d = h->d;
    launch_gauge_basis(d, h->stream);
    check_launch("gauge basis");
    std::vector<double> col((size_t)COARSE_GAUGE * d.nA);
    HIPCHK(hipMemcpyAsync(col.data(), d.Zc, col.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    sync(h);
    for (int e = 0; e < d.nA; ++e)
      for (int c = 0; c < COARSE_GAUGE; ++c) G[(size_t)e * COARSE_GAUGE + c] = col[(size_t)c * d.nA + e];
  });
}

ba_status ba_export_schur_dense(ba_handle* h, double* S) {
  if (!h || !S) return BA_E_INVALID;
  return guard(h, [&] {
    if (!h->finalized) throw BaError(BA_E_STATE, "no linearisation yet");
    set_device(h);
    const Dev& d = h->d;
    const size_t bytes = (size_t)d.nA * d.nA * sizeof(double);
    if (bytes == 0) return;
    double* Sd = nullptr;
    HIPCHK(hipMalloc((void**)&Sd, bytes));
    try {
      launch_dense_schur(d, h->last_lambda, Sd, h->stream);
      check_launch("dense reduced system");
      HIPCHK(hipMemcpyAsync(S, Sd, bytes, hipMemcpyDeviceToHost, h->stream));
      sync(h);
    } catch (...) {
      (void)hipFree(Sd);
      throw;
    }
    HIPCHK(hipFree(Sd));
  });
}

ba_status ba_export_schur_assembled(ba_handle* h, double* S) {
  if (!h || !S) return BA_E_INVALID;
  return guard(h, [&] {
    if (!h->finalized) throw BaError(BA_E_STATE, "no linearisation yet");
    set_device(h);
    dense_prepare(h);
    const Dev& d = h->d;
    if (d.nA == 0) return;
    launch_dense_assemble(d, h->last_lambda, h->stream);
    check_launch("dense assembly");
    HIPCHK(hipMemcpy2DAsync(S, (size_t)d.nA * 8, d.dS, (size_t)d.dense_npad * 8, (size_t)d.nA * 8, d.nA,
                            hipMemcpyDeviceToHost, h->stream));
    sync(h);
  });
}

ba_status ba_dense_spd_solve(int32_t device, int64_t n, double* A, double* b, void* hip_stream, int32_t* info) {
  if (info) *info = 0;
  if (n < 0 || (n > 0 && (!A || !b))) return BA_E_INVALID;
  if (n == 0) return BA_OK;
  int hinfo = 0;
  const ba_status st = guard(nullptr, [&] {
    if (n > (int64_t)1 << 20) throw BaError(BA_E_INVALID, "matrix too large");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) throw BaError(BA_E_INVALID, "bad device index");
    HIPCHK(hipSetDevice(device));
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t npad = (n + DENSE_NB - 1) / DENSE_NB * DENSE_NB;
    DevAlloc tmp;
    struct Release {
      DevAlloc& a;
      ~Release() { a.free_all(); }
    } release{tmp};
    double* Ap = tmp.get<double>((size_t)npad * npad);
    double* Linv = tmp.get<double>((size_t)npad * DENSE_NB);
    double* v = tmp.get<double>(npad);
    double* w = tmp.get<double>(npad);
    int* dinfo = tmp.get<int>(1);
    launch_dense_pad_identity(Ap, (int)n, (int)npad, s);
    HIPCHK(hipMemcpy2DAsync(Ap, npad * 8, A, n * 8, n * 8, n, hipMemcpyDeviceToDevice, s));
    launch_dense_zero_upper(Ap, (int)npad, s);
    launch_zero(v, npad * 8, s);
    launch_zero(dinfo, sizeof(int), s);
    HIPCHK(hipMemcpyAsync(v, b, n * 8, hipMemcpyDeviceToDevice, s));
    launch_dense_factor_solve(Ap, (int)npad, Linv, v, w, dinfo, s);
    check_launch("dense SPD solve");
    HIPCHK(hipMemcpy2DAsync(A, n * 8, Ap, npad * 8, n * 8, n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(b, v, n * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(&hinfo, dinfo, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  });
  if (st != BA_OK) return st;
  if (info) *info = hinfo;
  return hinfo ? BA_E_NUMERIC : BA_OK;
}

ba_status ba_export_schur_dense_noalloc(ba_handle* h, double* S) {
  if (!h || !S) return BA_E_INVALID;
  return guard(h, [&] {
    if (!h->finalized) throw BaError(BA_E_STATE, "no linearisation yet");
    set_device(h);
    const Dev& d = h->d;
    if (d.nA == 0) return;
    if (d.nA > NOALLOC_SCRATCH_DOUBLES)
      throw BaError(BA_E_INVALID, "reduced dimension " + std::to_string(d.nA) + " exceeds the no-allocation limit of " +
                                      std::to_string(NOALLOC_SCRATCH_DOUBLES));
    double* panel = noalloc_scratch(h->device);
    const int cols = (int)std::min<int64_t>(NOALLOC_SCRATCH_DOUBLES / d.nA, d.nA);
    for (int c0 = 0; c0 < d.nA; c0 += cols) {
      const int nc = std::min(cols, d.nA - c0);
      launch_dense_schur_columns(d, h->last_lambda, c0, nc, panel, h->stream);
      check_launch("dense reduced system (no allocation)");
      HIPCHK(hipMemcpyAsync(S + (int64_t)c0 * d.nA, panel, (size_t)nc * d.nA * sizeof(double), hipMemcpyDeviceToHost,
                            h->stream));
      sync(h);
    }
  });
}

ba_status ba_normalized_matvec(ba_handle* h, const double* x, double* y) {
  if (!h || !x || !y) return BA_E_INVALID;
  return guard(h, [&] {
    if (!h->finalized) throw BaError(BA_E_STATE, "no linearisation yet");
    set_device(h);
    const Dev& d = h->d;
    HIPCHK(hipMemcpyAsync(d.z, x, d.nA * 8, hipMemcpyHostToDevice, h->stream));
    ba_gnn_impl::launch_block_tri(d, d.z, d.p, true, h->stream);
    launch_schur_matvec(d, d.p, d.q, h->last_lambda, h->stream);
    ba_gnn_impl::launch_block_tri(d, d.q, d.z, false, h->stream);
    check_launch("normalized product");
    HIPCHK(hipMemcpyAsync(y, d.z, d.nA * 8, hipMemcpyDeviceToHost, h->stream));
    sync(h);
  });
}

const char* ba_last_error(const ba_handle* h) { return h ? h->err.c_str() : "null handle"; }

void ba_destroy(ba_handle* h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->gnn) ba_gnn_impl::destroy(h->gnn);
  h->alloc.free_all();
  if (h->hscal) (void)hipHostFree(h->hscal);
  if (h->events)
    for (int k = 0; k <= BA_PHASE_COUNT; ++k) (void)hipEventDestroy(h->ev[k]);
  for (hipEvent_t e : h->mv_ev) (void)hipEventDestroy(e);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

}  // extern "C"
