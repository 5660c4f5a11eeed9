// Launchers and registry of the systems emitted by the compiler slice from
// declared conservation laws (gen_systems.hpp, generated at build time).
#include "step_kernels.hpp"
#include "gen_systems.hpp"

namespace {

template <class Sys>
const Launchers *gen_launchers(int lat, int storage)
{
    if constexpr (Sys::D == 2) {
        if (lat == LAT_D2Q5) return by_storage<Sys, D2Q5>(storage);
        if (lat == LAT_D2Q9) return by_storage<Sys, D2Q9>(storage);
    } else {
        if (lat == LAT_D3Q7) return by_storage<Sys, D3Q7>(storage);
    }
    return nullptr;
}

template <int I>
const Launchers *launchers_at(int gen, int lat, int storage)
{
    if constexpr (I < kGenCount) {
        if (gen == I) return gen_launchers<SysGenOf<I>>(lat, storage);
        return launchers_at<I + 1>(gen, lat, storage);
    } else {
        return nullptr;
    }
}

}  // namespace

const Launchers *lbm_launchers_gen(int gen, int lat, int storage) { return launchers_at<0>(gen, lat, storage); }
int lbm_gen_count() { return kGenCount; }
const char *lbm_gen_name(int gen) { return (gen >= 0 && gen < kGenCount) ? kGenInfo[gen].name : nullptr; }
int lbm_gen_fields(int gen, int *D, int *n_conserved, int *npar)
{
    const GenInfo &g = kGenInfo[gen];
    *D = g.D;
    *n_conserved = g.n_conserved;
    *npar = g.npar;
    return g.K;
}
const char *lbm_gen_param_name(int gen, int j) { return kGenInfo[gen].param[j]; }
double lbm_gen_param_default(int gen, int j) { return kGenInfo[gen].param_default[j]; }
double lbm_gen_reference(int gen, int k) { return kGenInfo[gen].Q0[k]; }
