// LDS-tiled MFMA half-step kernel for the 3-D dissipative full method, m = 3.
#include "hw_kernels.h"

bool hw_tiled_supported(int d, int m, int method, int precision)
{
    (void)d; (void)m; (void)method; (void)precision;
    return false;
}

hipError_t hw_launch_tiled(const TiledArgs& a, int precision, hipStream_t st)
{
    (void)a; (void)precision; (void)st;
    return hipErrorInvalidValue;
}
