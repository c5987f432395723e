// Host-only entry to the pool validator, for the sanitizer build of
// cvx_validate.cpp (the library's own entry point sits in the HIP part).
#include <string>

#include "cvx_internal.h"

extern "C" int san_validate_pool(const cvx_canvas_desc* desc, const cvx_node* nodes,
                                 uint64_t n_nodes, const void* leaves, uint64_t n_leaves) {
  std::string msg;
  return cvx::validate_pool(desc, nodes, n_nodes, leaves, n_leaves, nullptr, msg);
}
