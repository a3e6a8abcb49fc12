// leb_internal.hpp -- launchers shared between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "leb.h"

namespace leb {

int launch_pbh_chain(const leb_dynamics* dyn, int64_t units, const double* z, const double* v,
                     const double* mu, const double* sigma, double* r_lo, double* r_hi, double* c_bar,
                     double* rho_bar, double pad, uint32_t* flags, hipStream_t stream,
                     const uint32_t* open = nullptr);
int launch_fill_zero(int64_t count, double* r_lo, double* r_hi, double* c_bar, double* rho_bar, double pad,
                     uint32_t* flags, int64_t nflags, hipStream_t stream);
size_t pbh_smem_bytes(int U);
size_t bwd_smem_bytes(int U);
int launch_tube_map(int B, int N, int U, const double* phi, const double* e, const double* cbar,
                    const double* rbar, double* mu, double* sigma, hipStream_t s);

// argument checks shared by the entry points
bool aligned8(const void* p);
int check_chain_dynamics(const leb_dynamics* dyn);

}  // namespace leb
