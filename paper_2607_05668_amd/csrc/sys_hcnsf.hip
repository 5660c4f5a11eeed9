// Launchers of the 3D homogenized compressible NSF system with the
// strain-reduced tracker basis (D3Q7, all storages).
#include "step_kernels.hpp"

const Launchers *lbm_launchers_hcnsf(int lat, int storage)
{
    return lat == LAT_D3Q7 ? by_storage<SysHCNSF, D3Q7>(storage) : nullptr;
}
