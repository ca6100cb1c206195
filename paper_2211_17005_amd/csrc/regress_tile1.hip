// The regression kernels in wave tiling variant 1: four output tiles by one row tile per wave (forward, back-propagation) and two input
// tiles per weight-gradient block.
#define HSIM_MLP_TILE 1
#include "regress.hip"
