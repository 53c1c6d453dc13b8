// Device helpers shared by the kernels that evaluate the basis at the points
// of an adaptive rule (Sec. IV.C): the shared table layout, the points of a
// slot's leaf boxes, the 1D Lagrange basis, the smooth cutoff of Eq. Moll1, the
// Slater-type radial terms and an atom's enrichment functions (Sec. IV.A-B).
#pragma once

#include "cf_kernels.h"

namespace cf {

// Shared tables (device array EnrAsm::tab): nodes [np1], Gauss x [ng] and w
// [ng] on [0, 1], then the shells: l [nsh], first term [nsh + 1], and the
// terms (c, k, zeta) [nterm].
struct EaTab {
  const double *nodes, *gx, *gw, *sl, *st, *terms;
};
__device__ __forceinline__ EaTab ea_tab(const double *s, const EnrAsm &a) {
  EaTab t;
  t.nodes = s;
  t.gx = t.nodes + a.np1;
  t.gw = t.gx + a.ng;
  t.sl = t.gw + a.ng;
  t.st = t.sl + a.nsh;
  t.terms = t.st + a.nsh + 1;
  return t;
}

// Point q of slot `slot`'s rule: coordinates, weight and potential.  Returns
// false past the slot's last point.
__device__ __forceinline__ bool ea_point(const EnrAsm &a, const EaTab &t, int slot, int64_t q,
                                         double x[3], double &w, double &v) {
  const int ng = a.ng, ng3 = ng * ng * ng;
  const int64_t b0 = a.bptr[slot], nb = a.bptr[slot + 1] - b0;
  if (q >= nb * ng3) return false;
  const int64_t b = b0 + q / ng3;
  const int r = (int)(q % ng3);
  const int ix = r % ng, iy = (r / ng) % ng, iz = r / (ng * ng);
  const double s = a.bsz[b];
  x[0] = a.blo[3 * b + 0] + s * t.gx[ix];
  x[1] = a.blo[3 * b + 1] + s * t.gx[iy];
  x[2] = a.blo[3 * b + 2] + s * t.gx[iz];
  w = s * s * s * (t.gw[ix] * t.gw[iy] * t.gw[iz]);
  v = a.V[b * ng3 + r];
  return true;
}

// Lagrange polynomials through the np1 nodes and their derivatives at s (the
// product over the other nodes; the derivative by the product rule).
__device__ __forceinline__ void ea_lagrange(const double *nodes, int np1, double s, double *L,
                                            double *dL) {
  for (int i = 0; i < np1; ++i) {
    double val = 1.0, der = 0.0;
    for (int j = 0; j < np1; ++j) {
      if (j == i) continue;
      const double inv = 1.0 / (nodes[i] - nodes[j]);
      const double f = (s - nodes[j]) * inv;
      der = der * f + val * inv;
      val *= f;
    }
    L[i] = val;
    dL[i] = der;
  }
}

// Smooth cutoff of Eq. Moll1 and its r-derivative:
//   r~ = 1 - t (r - r0) / r0, u(s) = exp(-1/s) (s > 0), h = u(r~) / (u(r~) + u(1 - r~)).
__device__ __forceinline__ void ea_cutoff(double r, double r0, double t, double &h, double &dh) {
  const double rt = 1.0 - t * (r - r0) / r0;
  if (rt >= 1.0) { h = 1.0; dh = 0.0; return; }
  if (rt <= 0.0) { h = 0.0; dh = 0.0; return; }
  const double a = exp(-1.0 / rt), b = exp(-1.0 / (1.0 - rt));
  const double da = a / (rt * rt), db = b / ((1.0 - rt) * (1.0 - rt));
  const double den = a + b;
  h = a / den;
  dh = (da * b + a * db) / (den * den) * (-t / r0);
}

// sum over a shell's terms of c r^(k - shift) exp(-zeta r) and its derivative
__device__ __forceinline__ void ea_radial(const EaTab &t, int sh, double r, int shift, double &v,
                                          double &dv) {
  v = 0.0;
  dv = 0.0;
  const int k0 = (int)t.st[sh], k1 = (int)t.st[sh + 1];
  for (int k = k0; k < k1; ++k) {
    const double c = t.terms[3 * k], z = t.terms[3 * k + 2];
    const int p = (int)t.terms[3 * k + 1] - shift;
    const double e = c * exp(-z * r);
    double pk = 1.0, pk1 = 0.0;                      // r^p and p r^(p-1)
    for (int i = 0; i < p; ++i) { pk1 = pk1 * r + pk; pk *= r; }
    v += pk * e;
    dv += (pk1 - z * pk) * e;
  }
}

// Values and gradients of atom I's npa functions at x, written to columns
// col0.. of the four LDS rows ev[0..3] (value, d/dx, d/dy, d/dz).
__device__ inline void ea_atom(const EnrAsm &a, const EaTab &t, int I, const double x[3], double *e0,
                        double *e1, double *e2, double *e3, int col0) {
  const double dx = x[0] - a.centers[3 * I], dy = x[1] - a.centers[3 * I + 1],
               dz = x[2] - a.centers[3 * I + 2];
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double rs = r > 1e-300 ? r : 1e-300;
  double h, dh;
  ea_cutoff(r, a.r0, a.t, h, dh);
  const double d[3] = {dx, dy, dz};
  constexpr double Y00 = 0.28209479177387814347;   // 1 / sqrt(4 pi)
  constexpr double Y1 = 0.48860251190291992159;    // sqrt(3 / (4 pi))
  int k = col0;
  for (int sh = 0; sh < a.nsh; ++sh) {
    const int l = (int)t.sl[sh];
    if (l == 0) {
      double R, dR;
      ea_radial(t, sh, r, 0, R, dR);
      const double g = h * R, dg = dh * R + h * dR;
      const double gr = Y00 * dg / rs;
      e0[k] = Y00 * g;
      e1[k] = gr * dx;
      e2[k] = gr * dy;
      e3[k] = gr * dz;
      ++k;
    } else {
      double S, dS;                                 // S = R / r
      ea_radial(t, sh, r, 1, S, dS);
      const double q = h * S, dq = dh * S + h * dS;
      const int axes[3] = {1, 2, 0};
      for (int m = 0; m < 3; ++m) {
        const int ax = axes[m];
        const double f = Y1 * d[ax] * dq / rs;
        e0[k] = Y1 * d[ax] * q;
        e1[k] = f * dx + (ax == 0 ? Y1 * q : 0.0);
        e2[k] = f * dy + (ax == 1 ? Y1 * q : 0.0);
        e3[k] = f * dz + (ax == 2 ? Y1 * q : 0.0);
        ++k;
      }
    }
  }
}


// Values only of atom I's npa functions at x into e0[col0 ..].
__device__ inline void ea_atom_val(const EnrAsm &a, const EaTab &t, int I, const double x[3],
                                   double *e0, int col0) {
  const double dx = x[0] - a.centers[3 * I], dy = x[1] - a.centers[3 * I + 1],
               dz = x[2] - a.centers[3 * I + 2];
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  double h, dh;
  ea_cutoff(r, a.r0, a.t, h, dh);
  const double d[3] = {dx, dy, dz};
  constexpr double Y00 = 0.28209479177387814347;   // 1 / sqrt(4 pi)
  constexpr double Y1 = 0.48860251190291992159;    // sqrt(3 / (4 pi))
  int k = col0;
  for (int sh = 0; sh < a.nsh; ++sh) {
    double R, dR;
    if ((int)t.sl[sh] == 0) {
      ea_radial(t, sh, r, 0, R, dR);
      e0[k++] = Y00 * (h * R);
    } else {
      ea_radial(t, sh, r, 1, R, dR);                // R / r
      const double q = h * R;
      e0[k++] = Y1 * d[1] * q;
      e0[k++] = Y1 * d[2] * q;
      e0[k++] = Y1 * d[0] * q;
    }
  }
}

}  // namespace cf
