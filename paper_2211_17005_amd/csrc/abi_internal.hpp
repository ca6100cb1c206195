// Helpers shared by the C-ABI translation units (validation, errors, tables).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/hsim.h"
#include "sim.hpp"

namespace hsim {

int fail(int code, const char* fmt, ...);
int device_error(hipError_t e, const char* what);
int check_market(const hsim_market* m);
int check_grid(const hsim_grid* g);
int check_book(const hsim_portfolio* p, const hsim_market* m, const hsim_grid* g, int* q_out, int* P_out);
int check_precision(int precision);
int check_paths(int64_t path_begin, int64_t M);
int check_nb(int32_t n_b, const int32_t* nb_block, int32_t block_paths);
int device_table(const std::vector<unsigned char>& blob, void** out);
size_t align256(size_t x);
template <typename Real>
int build_sim_args(const hsim_market* m, const hsim_portfolio* p, const hsim_grid* g, uint64_t seed,
                   int64_t path_begin, int64_t M, int feature_mode, SimArgs<Real>& a);

}  // namespace hsim

// Workspace of the operations implemented outside abi.hip (0 for unknown operations).
size_t hsim_adjoint_workspace(int op, const hsim_market* m, const hsim_grid* g, int64_t M, int precision);
