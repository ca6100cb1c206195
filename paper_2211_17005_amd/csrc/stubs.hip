#include "abi_internal.hpp"
size_t hsim_adjoint_workspace(int, const hsim_market*, const hsim_grid*, int64_t, int) { return 0; }
