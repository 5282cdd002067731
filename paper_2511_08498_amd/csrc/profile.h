// Line profiles evaluated on the device in single precision.
//
//   Gaussian: peak-normalised exp(-x^2).
//   Voigt:    H(a, x) = Re w(x + i a), the HUM1WEI24 scheme of Sect. 3.2.1
//             with one more Humlicek region: with s = |x| + a,
//               s > 15:        w ~ i z / (sqrt(pi) (z^2 - 1/2))          (region I)
//               5.5 <= s <= 15: w ~ t (1.410474 + 0.5641896 u) /
//                               (0.75 + u (3 + u)), t = a - i x, u = t^2 (region II)
//               s < 5.5:       the 24-term Weideman series (FMA Horner form).
//             Measured against the exact Faddeeva function (FP64): region II
//             is within 5.3e-5 relative, regions I and III within 8.4e-5 and
//             2.6e-5; region II costs ~25 VALU instead of ~125.  Each region's
//             one division is a multiplication by the hardware reciprocal
//             (1 ulp; a correctly rounded division costs ~10 VALU more, for
//             nothing measurable against the scheme's 1e-5 - 1e-4 error).
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
        return rsqrtpi * (nr * qr + ni * qi) * __builtin_amdgcn_rcpf(den);
    }
    if (s >= 5.5f) {
        // t = a - i x, u = t^2; w ~ t (A + B u) / (0.75 + u (3 + u))
        const float tr = a, ti = -x;
        const float ur = tr * tr - ti * ti, ui = 2.0f * tr * ti;
        const float pr = fmaf(0.5641896f, ur, 1.410474f), pim = 0.5641896f * ui;  // A + B u
        const float nr = tr * pr - ti * pim, ni = tr * pim + ti * pr;               // t (A + B u)
        const float vr = ur + 3.0f, vi = ui;                                         // 3 + u
        const float dr = 0.75f + (ur * vr - ui * vi), di = ur * vi + ui * vr;        // 0.75 + u (3 + u)
        return (nr * dr + ni * di) * __builtin_amdgcn_rcpf(dr * dr + di * di);
    }
    constexpr float c[24] = {RT_WEID_COEFS};
    const float Lw = RT_WEID_L;
    // i z = -a + i x;  L - i z = (L + a) - i x;  L + i z = (L - a) + i x
    float dr = Lw + a, di = -x;
    float nr = Lw - a, ni = x;
    float inv = __builtin_amdgcn_rcpf(dr * dr + di * di);
    float Zr = (nr * dr + ni * di) * inv;
    float Zi = (ni * dr - nr * di) * inv;
    // p(Z) = sum_k c_k Z^k has real coefficients: divided by the real quadratic (t - Z)(t - conj Z) =
    // t^2 - 2 Re Z t + |Z|^2 it leaves a remainder b1 t + b0, so p(Z) = Z b1 + (c_0 - |Z|^2 b2) with the
    // second-order recurrence b_k = c_k + 2 Re Z b_{k+1} - |Z|^2 b_{k+2} (Horner's scheme for a complex
    // argument, Knuth, TAOCP vol. 2, 4.6.4): two real FMAs per coefficient instead of a complex multiply-add.
    const float tz = 2.0f * Zr, m2 = fmaf(Zr, Zr, Zi * Zi);
    float b2 = 0.0f, b1 = c[23];
#pragma unroll
    for (int k = 22; k >= 1; --k) {
        const float b0 = fmaf(tz, b1, fmaf(-m2, b2, c[k]));
        b2 = b1;
        b1 = b0;
    }
    const float pr = fmaf(Zr, b1, fmaf(-m2, b2, c[0])), pi = Zi * b1;
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
