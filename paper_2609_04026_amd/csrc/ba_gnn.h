// Learned block-Jacobi correction: a small message-passing network over the
// camera / group covisibility graph of the reduced system.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "ba_internal.h"

namespace ba_gnn {
struct Net;
Net* create();
void destroy(Net* n);
bool load(Net* n, const void* blob, size_t bytes, hipStream_t s, std::string& err);
bool ready(const Net* n);
// build the graph of the problem (once per problem)
void attach(Net* n, const ba::Dev& d, hipStream_t s);
// overwrite the preconditioner blocks of d with the learned ones
void apply(Net* n, const ba::Dev& d, double lambda, hipStream_t s);
}  // namespace ba_gnn
