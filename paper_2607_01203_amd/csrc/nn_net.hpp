// nn_net.hpp -- the device copy of a ReLU MLP (the leb_mlp handle), shared by
// the bound (nn.hip) and its adjoint (nn_bwd.hip).
#pragma once
#include <vector>

namespace leb {
constexpr int NN_MAXW = 256;     // widest layer handled
constexpr int NN_MAXL = 8;       // most linear layers handled
}  // namespace leb

struct leb_mlp_s {
    int L;                          // linear layers
    int w[leb::NN_MAXL + 1];        // widths, w[0] inputs ... w[L] outputs
    int nx, nu, residual;
    double* W[leb::NN_MAXL];        // device, layer l+1: [w[l+1]][w[l]]
    double* WT[leb::NN_MAXL];       // device, transposed [w[l]][w[l+1]]
    double* b[leb::NN_MAXL];        // device [w[l+1]]
    std::vector<void*> allocs;
};
