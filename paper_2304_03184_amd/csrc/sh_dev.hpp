// Real spherical harmonics of a unit direction, bands l < degree (degree^2
// coefficients, l-major, m = -l..l), standard real basis:
//   Y_0 = 1/(2 sqrt(pi)),  Y_1 = sqrt(3/(4 pi)) (y, z, x), ...
#pragma once
#include <hip/hip_runtime.h>

namespace nvr {

__device__ __forceinline__ void sh_eval(float x, float y, float z, int degree, float *out) {
    // constants: sqrt of the normalisations of the real basis
    const float k00 = 0.28209479177387814f;          // 1/(2 sqrt(pi))
    const float k1 = 0.48860251190291992f;           // sqrt(3/(4 pi))
    const float k2a = 1.0925484305920790f;           // (1/2) sqrt(15/pi)
    const float k20 = 0.31539156525252005f;          // (1/4) sqrt(5/pi)
    const float k22 = 0.54627421529603959f;          // (1/4) sqrt(15/pi)
    const float k3a = 0.59004358992664352f;          // (1/4) sqrt(35/(2 pi))
    const float k3b = 2.8906114426405538f;           // (1/2) sqrt(105/pi)
    const float k3c = 0.45704579946446572f;          // (1/4) sqrt(21/(2 pi))
    const float k30 = 0.37317633259011540f;          // (1/4) sqrt(7/pi)
    const float k3d = 1.4453057213202769f;           // (1/4) sqrt(105/pi)
    out[0] = k00;
    if (degree <= 1) return;
    out[1] = k1 * y;
    out[2] = k1 * z;
    out[3] = k1 * x;
    if (degree <= 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    out[4] = k2a * x * y;
    out[5] = k2a * y * z;
    out[6] = k20 * (3.f * zz - 1.f);
    out[7] = k2a * x * z;
    out[8] = k22 * (xx - yy);
    if (degree <= 3) return;
    out[9] = k3a * y * (3.f * xx - yy);
    out[10] = k3b * x * y * z;
    out[11] = k3c * y * (5.f * zz - 1.f);
    out[12] = k30 * z * (5.f * zz - 3.f);
    out[13] = k3c * x * (5.f * zz - 1.f);
    out[14] = k3d * z * (xx - yy);
    out[15] = k3a * x * (xx - 3.f * yy);
}

}  // namespace nvr
