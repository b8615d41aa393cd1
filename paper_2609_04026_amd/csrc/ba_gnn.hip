// Learned block-Jacobi correction (network kernels).
#include "ba_gnn.h"

namespace ba_gnn {
struct Net {
  bool loaded = false;
};
Net* create() { return new Net(); }
void destroy(Net* n) { delete n; }
bool load(Net* n, const void*, size_t, hipStream_t, std::string& err) {
  err = "learned preconditioner weights are not supported by this build";
  n->loaded = false;
  return false;
}
bool ready(const Net* n) { return n && n->loaded; }
void attach(Net*, const ba::Dev&, hipStream_t) {}
void apply(Net*, const ba::Dev&, double, hipStream_t) {}
}  // namespace ba_gnn
