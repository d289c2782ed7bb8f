// Entry points that are declared in iat.h but not yet implemented in this build.
#include "iat_host.h"

using namespace iat;


extern "C" int iat_adjoint(const iat_system*, const iat_species*, int, const iat_batch*, const iat_obs*,
                           const double*, double*, const void*, size_t, void*, size_t, const iat_launch*, void*)
{
    return set_error(IAT_ENOTSUP, "iat_adjoint is not implemented yet");
}


extern "C" int iat_workspace_bytes(int, const iat_system*, const iat_batch*, size_t*)
{
    return set_error(IAT_ENOTSUP, "iat_workspace_bytes is not implemented yet");
}
