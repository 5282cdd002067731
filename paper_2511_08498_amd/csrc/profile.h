// Line profiles evaluated on the device in single precision.
//
//   Gaussian: peak-normalised exp(-x^2).
//   Voigt:    H(a, x) = Re w(x + i a) by the HUM1WEI24 scheme (Sect. 3.2.1):
//             Humlicek's region-I rational approximation
//             w ~ i z / (sqrt(pi) (z^2 - 1/2)) where |x| + a > 15, and the
//             24-term Weideman series elsewhere (FMA-friendly Horner form).
//             phi = H / (sqrt(pi) dlD); eta*, chi* carry lam0/lam and the
//             damping (lam/lam0)^2 (Sect. 3.2.1 wavelength scalings).
#pragma once

#include <hip/hip_runtime.h>

#include "weideman24.h"

namespace rt {

__device__ __forceinline__ float voigt_h(float a, float x)
{
    const float rsqrtpi = 0.56418958354775628f;
    float s = fabsf(x) + a;
    if (s > 15.0f) {
        // z = x + i a;  w = i z / (sqrt(pi) (z^2 - 1/2)),  H = Re w
        float zr = x, zi = a;
        float qr = zr * zr - zi * zi - 0.5f, qi = 2.0f * zr * zi;  // z^2 - 1/2
        float nr = -zi, ni = zr;                                    // i z
        float den = qr * qr + qi * qi;
        return rsqrtpi * (nr * qr + ni * qi) / den;
    }
    constexpr float c[24] = {RT_WEID_COEFS};
    const float Lw = RT_WEID_L;
    // i z = -a + i x;  L - i z = (L + a) - i x;  L + i z = (L - a) + i x
    float dr = Lw + a, di = -x;
    float nr = Lw - a, ni = x;
    float inv = 1.0f / (dr * dr + di * di);
    float Zr = (nr * dr + ni * di) * inv;
    float Zi = (ni * dr - nr * di) * inv;
    float pr = c[23], pi = 0.0f;
#pragma unroll
    for (int k = 22; k >= 0; --k) {
        float tr = fmaf(pr, Zr, fmaf(-pi, Zi, c[k]));
        pi = fmaf(pr, Zi, pi * Zr);
        pr = tr;
    }
    // 1/(L - i z) and its square
    float ir = dr * inv, ii = -di * inv;
    float i2r = ir * ir - ii * ii, i2i = 2.0f * ir * ii;
    return 2.0f * (pr * i2r - pi * i2i) + rsqrtpi * ir;
}

// Factor multiplying eta*, chi* of one line: Gaussian exp(-x^2), or the Voigt
// profile with the wavelength scalings.  x = (lam - lam0 (1 - u/c)) / dlD.
__device__ __forceinline__ float line_shape(int profile, float x, float a0, double lam, double lam0, float inv_dld)
{
    if (profile == RT_PROFILE_GAUSS) return __expf(-x * x);
    const float rsqrtpi = 0.56418958354775628f;
    float r = (float)(lam / lam0);
    float H = voigt_h(a0 * r * r, x);
    return H * inv_dld * rsqrtpi / r;
}

}  // namespace rt
