// Learned coarse-space correction of the PCG preconditioner: a small
// message-passing network over the camera / group graph of the reduced
// system (definitions in ba_gnn.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "ba_internal.h"
#include "ba_math.h"

struct ba_gnn;

namespace ba_gnn_impl {

constexpr int NODE_IN = 64, EDGE_IN = 8, HEAD_PAD = 9 * ba::COARSE_NET;
constexpr int MAX_GRAPH_NODES = 6000;  // the symbolic phase counts shared features in a dense n x n table

// host-side graph of a problem's reduced system, built once at the symbolic phase
struct Graph {
  int n_nodes = 0, n_edges = 0;
  std::vector<int32_t> node_type, node_off, node_size, edge_src, edge_dst, edge_rev, dst_off;
  std::vector<float> node_static;  // n x 64: the structural input entries (others zero)
  std::vector<float> edge_x;       // m x 8
  std::vector<int2> edge_typed;    // m: (bits of edge_x[0], index 1..4 of its one-hot kind column)
  double scale = 1.0;              // scene scale s0 (RMS camera-centre spread of the input cameras)
  bool valid = false;
};

// nodes ordered cameras, planes, VPs; feature f touches blocks fb[fb_off[f] .. fb_off[f+1])
// (distinct); block_records: records per block
void build_graph(Graph& g, int nc, int ng, int nv, int cd, const std::vector<int64_t>& fb_off,
                 const std::vector<int32_t>& fb, const std::vector<int64_t>& block_records, double scale);

// node input features (n x 64, device) from the structural entries, the
// damped diagonal blocks of S and the current geometry (lengths over s0)
void launch_node_features(const ba::Dev& d, const float* stat, const int32_t* type, int n, double lambda, double s0,
                          float* out, hipStream_t s);
// y = L^-1 v (transposed = false) or L^-T v (true) blockwise, S_ii = L_i L_i^T
void launch_block_tri(const ba::Dev& d, const double* v, double* y, bool transposed, hipStream_t s);

ba_gnn* create(int cd, int precision, int device, std::string& err);
void destroy(ba_gnn* n);
bool load(ba_gnn* n, const void* blob, size_t bytes, std::string& err);
// weights loaded and a graph attached
bool ready(const ba_gnn* n);
// upload the problem graph (once per problem)
void attach(ba_gnn* n, const Graph& g);
// write the coarse basis d.Zc from the network (ordered on s); the caller
// then forms E = Z^T S Z (launch_coarse_setup)
void apply(ba_gnn* n, const ba::Dev& d, double lambda, hipStream_t s);
size_t param_count(int cd);

}  // namespace ba_gnn_impl
