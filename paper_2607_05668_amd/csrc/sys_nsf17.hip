// Launchers of the 3D compressible NSF cascade with 12 trackers (D3Q7, all
// storages).
#include "step_kernels.hpp"

const Launchers *lbm_launchers_nsf17(int lat, int storage)
{
    return lat == LAT_D3Q7 ? by_storage<SysNSF17, D3Q7>(storage) : nullptr;
}
