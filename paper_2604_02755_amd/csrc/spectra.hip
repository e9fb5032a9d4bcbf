// Velocity response spectra of receiver records (Section 3).
#include <hip/hip_runtime.h>

#include <cmath>

#include "nlth_impl.hpp"

namespace nlth {

// ---------------------------------------------------------------------------
// velocity response spectra of receiver records (Section 3, h = 0.05)
// ---------------------------------------------------------------------------

// One thread per (series, period), periods fastest (the threads of a series
// read the same samples).  The ground velocity is linear between samples, so
// the ground acceleration a_n = (v_n - v_{n-1}) / dt is constant on a step;
// over a step the oscillator x'' + 2 h w x' + w^2 x = -a moves as free damped
// vibration about its static offset -a / w^2, which gives the exact update
//   y = x + a / w^2,  y(dt) = E ((C + q S) y + (S / wd) x'),
//   x'(dt) = E (-(w / r) S y + (C - q S) x'),  x(dt) = y(dt) - a / w^2,
// with wd = w r, r = sqrt(1 - h^2), q = h / r, E = exp(-h w dt),
// C = cos(wd dt), S = sin(wd dt).
__global__ void k_response_spectra(const double* __restrict__ vel, int ns, int nt, double dt,
                                   const double* __restrict__ periods, int np, double h, int kind,
                                   double* __restrict__ out)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)ns * np) return;
    const int sr = (int)(t / np), pk = (int)(t % np);
    const double w = 2.0 * M_PI / periods[pk];
    const double r = sqrt(1.0 - h * h), wd = w * r, q = h / r;
    const double E = exp(-h * w * dt), C = cos(wd * dt), S = sin(wd * dt);
    const double a11 = E * (C + q * S), a12 = E * S / wd, a21 = -E * w * S / r, a22 = E * (C - q * S);
    const double iw2 = 1.0 / (w * w), idt = 1.0 / dt;
    const double* v = vel + (size_t)sr * nt;
    double x = 0.0, xd = 0.0, vp = 0.0, px = 0.0, pv = 0.0;
    for (int n = 0; n < nt; ++n) {
        const double vn = v[n];
        const double off = (vn - vp) * idt * iw2;  // a_n / w^2
        vp = vn;
        const double y = x + off;
        const double y1 = a11 * y + a12 * xd;
        xd = a21 * y + a22 * xd;
        x = y1 - off;
        px = fmax(px, fabs(x));
        pv = fmax(pv, fabs(xd));
    }
    out[t] = kind == 0 ? pv : w * px;
}

void launch_response_spectra(hipStream_t s, const double* vel, int ns, int nt, double dt, const double* periods, int np,
                             double h, int kind, double* out)
{
    const long n = (long)ns * np;
    if (n > 0) hipLaunchKernelGGL(k_response_spectra, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, vel, ns, nt, dt, periods, np, h,
                                  kind, out);
}

}  // namespace nlth
