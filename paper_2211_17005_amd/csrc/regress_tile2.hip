// The regression kernels in wave tiling variant 2: one output tile by four row tiles per wave (forward, back-propagation) and every input
// tile of a weight-gradient row per block.
#define HSIM_MLP_TILE 2
#include "regress.hip"
