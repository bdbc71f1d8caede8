// Generalized plasmon-pole extension of the static inverse dielectric matrix to real
// frequencies (the frequency model the paper's calculations use):
//   Omega^2_{GG'} = w_p^2 [(q+G).(q+G') / |q+G|^2] rho(G - G') / rho(0),  w_p^2 = 4 pi rho(0)
//   wt^2_{GG'}    = Omega^2_{GG'} / (delta_{GG'} - eps^-1_{GG'}(0))
//   eps^-1_{GG'}(w) = delta_{GG'} + Omega^2_{GG'} / ((w + i eta)^2 - wt^2_{GG'})
// An element with delta - eps^-1(0) = 0 (unscreened) has no pole and keeps its static value.
// One thread per (G, G'): HBM-bound (reads eps^-1(0) once, writes every frequency).
#include "common.h"
#include "internal.h"

namespace gw {

namespace {

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  // scaled complex division (Smith's method)
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + r * b.y;
    return double2{(a.x + a.y * r) / d, (a.y - a.x * r) / d};
  }
  const double r = b.x / b.y, d = b.y + r * b.x;
  return double2{(a.x * r + a.y) / d, (a.y * r - a.x) / d};
}

__global__ void k_gpp(const double2* __restrict__ eps0, int ng, const double* __restrict__ kvec,
                      const int32_t* __restrict__ gvec, const double2* __restrict__ rho, int half,
                      const double* __restrict__ omega, int nomega, double eta, double2* __restrict__ modes,
                      double2* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n2 = (size_t)ng * ng;
  if (e >= n2) return;
  const int a = (int)(e / ng), b = (int)(e % ng);
  const double* ka = kvec + 3 * a;
  const double* kb = kvec + 3 * b;
  const double dot = ka[0] * kb[0] + ka[1] * kb[1] + ka[2] * kb[2];
  const double nrm = ka[0] * ka[0] + ka[1] * ka[1] + ka[2] * ka[2];
  const int w = 2 * half + 1;
  const int d0 = gvec[3 * a] - gvec[3 * b] + half, d1 = gvec[3 * a + 1] - gvec[3 * b + 1] + half,
            d2 = gvec[3 * a + 2] - gvec[3 * b + 2] + half;
  const double2 r = rho[((size_t)d0 * w + d1) * w + d2];   // the host checked the box covers G - G'
  const double s = 4.0 * M_PI * dot / nrm;                 // w_p^2 rho(G - G') / rho(0) = 4 pi rho(G - G')
  const double2 om2{s * r.x, s * r.y};
  const double2 z0 = eps0[e];
  const double2 den{(a == b ? 1.0 : 0.0) - z0.x, -z0.y};
  const bool pole = den.x != 0.0 || den.y != 0.0;
  const double2 wt2 = pole ? cdiv(om2, den) : double2{INFINITY, 0.0};
  if (modes) {
    modes[e] = om2;
    modes[n2 + e] = wt2;
  }
  for (int i = 0; i < nomega; ++i) {
    double2 v{a == b ? 1.0 : 0.0, 0.0};
    if (pole) {
      const double wr = omega[i];
      const double2 zz{wr * wr - eta * eta - wt2.x, 2.0 * wr * eta - wt2.y};   // (w + i eta)^2 - wt^2
      const double2 t = cdiv(om2, zz);
      v.x += t.x;
      v.y += t.y;
    } else {
      v = z0;
    }
    out[(size_t)i * n2 + e] = v;
  }
}

}  // namespace

hipError_t launch_gpp(const void* eps0, int ng, const double* kvec, const int32_t* gvec, const void* rho, int half,
                      const double* omega, int nomega, double eta, void* modes, void* out, hipStream_t st) {
  const size_t n = (size_t)ng * ng;
  k_gpp<<<(unsigned)((n + 255) / 256), 256, 0, st>>>((const double2*)eps0, ng, kvec, gvec, (const double2*)rho, half,
                                                     omega, nomega, eta, (double2*)modes, (double2*)out);
  return hipGetLastError();
}

}  // namespace gw
