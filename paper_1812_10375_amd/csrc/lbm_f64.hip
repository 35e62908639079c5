// FP64 instantiation.  This file is compiled with -ffp-contract=off: together with
// the plain-order code paths selected for double in lbm_kernels.hpp it rounds every
// operation as written.
#include "lbm_launch.hpp"
LBM_INSTANTIATE(double)
