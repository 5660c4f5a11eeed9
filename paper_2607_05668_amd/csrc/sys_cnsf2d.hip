// Launchers of 2D compressible Navier-Stokes-Fourier (all storages, D2Q5 and D2Q9).
#include "step_kernels.hpp"

LBM_DEFINE_LAUNCHERS_2D(lbm_launchers_cnsf2d, SysCNSF2D)
