// FP32 instantiation of the kernels and launches (populations, temperature, rho and u
// in FP32; equation of state and all reductions in FP64).
#include "lbm_launch.hpp"
LBM_INSTANTIATE(float)
