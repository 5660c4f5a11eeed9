// Launchers of 2D resistive compressible MHD (all storages, D2Q5 and D2Q9).
#include "step_kernels.hpp"

LBM_DEFINE_LAUNCHERS_2D(lbm_launchers_mhd, SysMHD)
