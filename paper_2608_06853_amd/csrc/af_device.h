// Device-side building blocks shared by the HIP kernels of the library:
// the two-layer lens refraction (Fermat's principle, Eqs. 7-8), the Keys
// bicubic weights and the trapezoid path sum of the slowness deviation
// (Eq. 1 discretised as in Section III-A).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace af {

constexpr int TILE = 256;           // points per tile = threads of a DAS workgroup
constexpr int SUB = 64;             // points per CMPE sub-tile = one wavefront

// One travel-time table entry: sample position u = ui + uf of (T + t_ttp/2 - t0/2) * fs
// and the apodised phasor h * exp(j 2 pi fd (T + t_ttp/2)).  A masked entry (h = 0)
// has ui = 0, uf = 0 and a zero phasor, so its samples contribute nothing.
struct alignas(16) TabEntry {
  int ui;
  float uf;
  float er, ei;
};

// 1/sqrt(x) and 1/x in FP64: the hardware estimate refined by one Newton step
// (relative error below 2^-44, far inside what a travel time needs).
__device__ inline double rsqrt64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x * y;
  return fma(y, fma(-h, y, 0.5), y);
}
__device__ inline double rcp64(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return fma(y, fma(-x, y, 1.0), y);
}

struct RayOut {
  double t_hom;   // L1/c_lens + L2/c_med at the refraction point
  float refx;     // refraction point on the lens arc (global frame)
  float refz;
  float l2;       // medium leg length
};

// Fermat ray through the concentric lens.  Element: radius R, polar unit vector
// (sa, ca) = (sin, cos) of its polar angle.  Point: radius rho, polar unit vector
// (sp, cp).  icl, icm: 1/c_lens and 1/c_med.
//
// The stationary point of T is found in the local frame of the element (element
// on the z axis) by safeguarded FP32 Newton on the Snell residual
//   G(alpha) = sin(i1)/c_lens - sin(i2)/c_med,
// where alpha is the direction of the lens leg; G is close to linear in alpha.
// The iterations only place the start of the FP64 step, so they divide with the
// hardware reciprocal (1 ulp) instead of correctly rounded divisions.
// The lens point is then projected onto the arc in FP64 and one FP64 second-order
// step on T(phi) gives T at the stationary point (error O(dphi^3)) and the
// refined refraction point.
__device__ inline RayOut trace_lens(double R, double sa, double ca, double rho, double sp,
                                    double cp, double dlens, double icl, double icm) {
  if (dlens == 0.0) {
    // no lens: the ray runs straight from the element, which is its own refraction point
    const double ex = R * sa, ez = R * ca;
    const double vx = rho * sp - ex, vz = rho * cp - ez;
    const double L2 = sqrt(vx * vx + vz * vz);
    RayOut o;
    o.t_hom = L2 * icm;
    o.refx = (float)ex;
    o.refz = (float)ez;
    o.l2 = (float)L2;
    return o;
  }
  const double RL = R + dlens;
  const double cT = cp * ca + sp * sa;   // cos(theta_p - theta_a)
  double sT = sp * ca - cp * sa;         // sin(theta_p - theta_a)
  const double sgn = sT < 0.0 ? -1.0 : 1.0;
  sT = fabs(sT);

  const float Rf = (float)R;
  const float RLf = (float)RL;
  const float d2f = (float)((RL - R) * (RL + R));
  const float pxf = (float)(rho * sT);
  const float pzf = (float)(rho * cT);
  const float iclf = (float)icl, icmf = (float)icm;
  const float irl = (float)(1.0 / RL);

  float lo = 0.f;
  float hi = atan2f(pxf, pzf - Rf);   // straight direction from the element to the point
  // thin-lens guess: Snell at the lens apex above the element
  float vz0 = pzf - RLf;
  float si2g = pxf * rsqrtf(fmaxf(pxf * pxf + vz0 * vz0, 1e-30f));
  float si1g = fminf(fmaxf(si2g * (icmf / iclf), 0.f), 0.95f);
  float x = fminf(fmaxf(asinf(si1g), lo), hi);
  float lx = 0.f, lz = Rf + (float)(RL - R);
#pragma unroll
  // Two safeguarded Newton updates in FP32 with the hardware sine and cosine: the
  // FP64 step below converges quadratically from there, and T is stationary in the
  // refraction angle, so the time is exact to FP32 rounding.
  for (int it = 0; it < 3; ++it) {
    float s, c;
    s = __sinf(x);
    c = __cosf(x);
    const float Q = sqrtf(Rf * Rf * c * c + d2f);
    const float iQ = __builtin_amdgcn_rcpf(Q);
    const float L1 = d2f * __builtin_amdgcn_rcpf(Rf * c + Q);
    const float dL1 = Rf * s * L1 * iQ;
    lx = L1 * s;
    lz = Rf + L1 * c;
    const float dlx = dL1 * s + L1 * c;
    const float dlz = dL1 * c - L1 * s;
    const float nx = lx * irl, nz = lz * irl, dnx = dlx * irl, dnz = dlz * irl;
    const float si1 = s * nz - c * nx;
    const float dsi1 = (c * nz + s * nx) + (s * dnz - c * dnx);
    const float vx = pxf - lx, vz = pzf - lz;
    const float iL2 = rsqrtf(vx * vx + vz * vz);
    const float cr = vx * nz - vz * nx;
    const float dcr = (-dlx * nz + dlz * nx) + (vx * dnz - vz * dnx);
    const float vdv = -(vx * dlx + vz * dlz);
    const float si2 = cr * iL2;
    const float dsi2 = dcr * iL2 - cr * vdv * iL2 * iL2 * iL2;
    const float g = si1 * iclf - si2 * icmf;
    const float dg = dsi1 * iclf - dsi2 * icmf;
    if (it == 2) break;  // (lx, lz) is the lens point at the last alpha
    if (g < 0.f) lo = x; else hi = x;
    const float nw = x - g * __builtin_amdgcn_rcpf(dg);
    x = (nw >= lo && nw <= hi) ? nw : 0.5f * (lo + hi);
  }

  // FP64: project onto the arc, one second-order step in phi
  const double lxd = lx, lzd = lz;
  const double inv = rsqrt64(lxd * lxd + lzd * lzd);
  const double s = lxd * inv, c = lzd * inv;       // sin, cos of phi'
  const double omc = s * s * rcp64(1.0 + c);       // 1 - cos(phi')
  const double dd = RL - R;
  const double l1sq = dd * dd + 2.0 * R * RL * omc;
  const double cw = cT * c + sT * s;               // cos(Theta - phi')
  const double sw = sT * c - cT * s;               // sin(Theta - phi')
  const double omw = cw > 0.0 ? sw * sw * rcp64(1.0 + cw) : 1.0 - cw;
  const double hh = rho - RL;
  const double l2sq = hh * hh + 2.0 * rho * RL * omw;
  const double i1 = rsqrt64(l1sq), i2 = rsqrt64(l2sq);
  const double L1 = l1sq * i1, L2 = l2sq * i2;
  const double d1 = R * RL * s * i1;
  const double d2 = -rho * RL * sw * i2;
  const double Tp = d1 * icl + d2 * icm;
  const double Tpp = (R * RL * c - d1 * d1) * i1 * icl + (rho * RL * cw - d2 * d2) * i2 * icm;
  const double del = Tpp > 0.0 ? -Tp * rcp64(Tpp) : 0.0;
  RayOut o;
  o.t_hom = L1 * icl + L2 * icm + 0.5 * Tp * del;
  // refined refraction point (first-order rotation by del) in the global frame
  const double cs = c - s * del, ss = (s + c * del) * sgn;
  o.refx = (float)(RL * (sa * cs + ca * ss));
  o.refz = (float)(RL * (ca * cs - sa * ss));
  o.l2 = (float)(L2 + d2 * del);
  return o;
}

// Discrete refraction search (Section III-A: the refraction point is the best of
// a finite set of N_search lens points, taken at the homogeneous mean speed).
// The candidates are n >= 2 lens points evenly spaced in polar angle over the
// interval that holds the minimiser of T: from the element's own polar angle to
// the point where the straight element-point segment crosses the lens arc when
// the lens is the slower layer (Snell bends the lens leg towards the normal),
// else from that crossing to the point's polar angle.  The candidate of least
// L1/c_lens + L2/c_med is taken, the first one on ties.  Same arguments and
// outputs as trace_lens; FP64 throughout.
__device__ inline RayOut trace_lens_search(double R, double sa, double ca, double rho, double sp,
                                           double cp, double dlens, double icl, double icm,
                                           int n) {
  const double RL = R + dlens;
  const double cT = cp * ca + sp * sa;
  double sT = sp * ca - cp * sa;
  const double sgn = sT < 0.0 ? -1.0 : 1.0;
  sT = fabs(sT);
  const double px = rho * sT, pz = rho * cT;  // point in the element's frame, element at (0, R)
  // crossing of the segment (0, R) -> (px, pz) with the arc of radius RL
  const double dz = pz - R;
  const double dd = px * px + dz * dz;
  const double ed = R * dz;
  double t = dd > 0.0 ? (-ed + sqrt(fmax(ed * ed + dd * (RL * RL - R * R), 0.0))) / dd : 0.0;
  t = fmin(fmax(t, 0.0), 1.0);
  const double phx = atan2(t * px, R + t * dz);
  const double lo = icl >= icm ? 0.0 : phx;
  const double hi = icl >= icm ? phx : atan2(px, pz);
  const double step = (hi - lo) / (double)(n - 1);
  double best = 1e300, bs = 0.0, bc = 1.0, bl2 = 0.0;
  for (int k = 0; k < n; ++k) {
    double s, c;
    sincos(lo + step * (double)k, &s, &c);
    const double lx = RL * s, lz = RL * c;
    const double l1 = sqrt(lx * lx + (lz - R) * (lz - R));
    const double l2 = sqrt((px - lx) * (px - lx) + (pz - lz) * (pz - lz));
    const double T = l1 * icl + l2 * icm;
    if (T < best) {
      best = T;
      bs = s;
      bc = c;
      bl2 = l2;
    }
  }
  RayOut o;
  o.t_hom = best;
  const double ss = bs * sgn;
  o.refx = (float)(RL * (sa * bc + ca * ss));
  o.refz = (float)(RL * (ca * bc - sa * ss));
  o.l2 = (float)bl2;
  return o;
}

// Fermat ray through a flat lens (linear array; Eqs. 7-8 with a plane interface).
// Element at (xe, ze); the lens is the layer ze <= z <= ze + dlens; point at
// (xp, zp) below it.  The lens point is (xe +- xi, ze + dlens) with lateral
// offset xi >= 0 towards the point.  T(xi) is convex; its minimiser lies between
// 0 and the straight crossing uc = u dlens / (zp - ze) when the lens is the slower
// layer, between uc and u otherwise.  FP64 Newton on dT/dxi from the thin-lens
// guess, safeguarded by bisection inside that bracket; with nsearch >= 2 the best
// of nsearch evenly spaced candidates over the same interval (the first on ties).
// dlens = 0 is the straight ray from the element.
__device__ inline RayOut trace_flat(double xe, double ze, double xp, double zp, double dlens,
                                    double icl, double icm, int nsearch) {
  const double dx = xp - xe;
  const double sgn = dx < 0.0 ? -1.0 : 1.0;
  const double u = fabs(dx);
  const double H = zp - ze;
  RayOut o;
  if (dlens == 0.0) {
    const double L2 = sqrt(u * u + H * H);
    o.t_hom = L2 * icm;
    o.refx = (float)xe;
    o.refz = (float)ze;
    o.l2 = (float)L2;
    return o;
  }
  const double h = H - dlens;  // depth of the point below the lens surface
  const double uc = H > 0.0 ? u * dlens / H : 0.0;
  const double lo = icl >= icm ? 0.0 : uc, hi = icl >= icm ? uc : u;
  const double d2 = dlens * dlens, h2 = h * h;
  double xi;
  if (nsearch >= 2) {
    const double step = (hi - lo) / (double)(nsearch - 1);
    double best = 1e300;
    xi = lo;
    for (int k = 0; k < nsearch; ++k) {
      const double x = lo + step * (double)k;
      const double T = sqrt(x * x + d2) * icl + sqrt((u - x) * (u - x) + h2) * icm;
      if (T < best) {
        best = T;
        xi = x;
      }
    }
  } else {
    double a = lo, b = hi;
    xi = icl >= icm ? uc * (icm / icl) : uc;
    for (int it = 0; it < 6; ++it) {
      const double L1 = sqrt(xi * xi + d2), L2 = sqrt((u - xi) * (u - xi) + h2);
      const double g = xi / L1 * icl - (u - xi) / L2 * icm;
      const double gp = d2 / (L1 * L1 * L1) * icl + h2 / (L2 * L2 * L2) * icm;
      if (g < 0.0) a = xi; else b = xi;
      const double nw = xi - g / gp;
      xi = (nw >= a && nw <= b) ? nw : 0.5 * (a + b);
    }
  }
  const double L1 = sqrt(xi * xi + d2), L2 = sqrt((u - xi) * (u - xi) + h2);
  o.t_hom = L1 * icl + L2 * icm;
  o.refx = (float)(xe + sgn * xi);
  o.refz = (float)(ze + dlens);
  o.l2 = (float)L2;
  return o;
}

// Refraction modes: the lens surface is the concentric arc (curvilinear array)
// or a plane (linear array), and the refraction point the continuous root or the
// discrete search.  Element descriptor: (R, sin, cos) of the element on the arc,
// or (x, z) on the line; point descriptor: (rho, sin, cos), or (x, z).
enum RefractMode { ARC_ROOT = 0, ARC_SEARCH = 1, FLAT_ROOT = 2, FLAT_SEARCH = 3 };

inline int refract_mode(bool flat, int nsearch, double dlens) {
  return (flat ? FLAT_ROOT : ARC_ROOT) + (nsearch >= 2 && dlens > 0.0 ? 1 : 0);
}

template <int MODE>
__device__ inline RayOut refract(const double4& el, const double4& pp, double dlens, double icl,
                                 double icm, int nsearch) {
  if (MODE == FLAT_ROOT || MODE == FLAT_SEARCH)
    return trace_flat(el.x, el.y, pp.x, pp.y, dlens, icl, icm, MODE == FLAT_SEARCH ? nsearch : 0);
  if (MODE == ARC_SEARCH)
    return trace_lens_search(el.x, el.y, el.z, pp.x, pp.y, pp.z, dlens, icl, icm, nsearch);
  return trace_lens(el.x, el.y, el.z, pp.x, pp.y, pp.z, dlens, icl, icm);
}

// Keys cubic-convolution weights (a = -0.5) of the taps at offsets -1, 0, 1, 2
// for fractional position f in [0, 1].
__device__ inline void keys_weights(float f, float& w0, float& w1, float& w2, float& w3) {
  const float f2 = f * f;
  w0 = f * (-0.5f + f * (1.0f - 0.5f * f));
  w1 = 1.0f + f2 * (-2.5f + 1.5f * f);
  w2 = f * (0.5f + f * (2.0f - 1.5f * f));
  w3 = f2 * (-0.5f + 0.5f * f);
}

// c times the Keys weights, c folded into the polynomials: c f and c f^2 take the
// place of f^2, so the scale costs one multiply instead of four.
__device__ inline void keys_weights_scaled(float f, float c, float& w0, float& w1, float& w2,
                                           float& w3) {
  const float cf = c * f, cf2 = cf * f;
  w0 = cf * fmaf(f, fmaf(-0.5f, f, 1.0f), -0.5f);
  w1 = fmaf(cf2, fmaf(1.5f, f, -2.5f), c);
  w2 = cf * fmaf(f, fmaf(-1.5f, f, 2.0f), 0.5f);
  w3 = cf2 * fmaf(0.5f, f, -0.5f);
}

// Trapezoid sum over k = 0..nseg of the bicubic value of a padded node grid at
// grid coordinates (u0 + k du, v0 + k dv), clamped to the node range.  The padded
// grid has row stride W = nx + 3 and holds node (i, j) at (i + 1) * W + (j + 1)
// for i in [-1, nz + 1], j in [-1, nx + 1] (edge values replicated).  Returns
// sum_k w_k value_k with w = 1/2 at both ends and 1 inside (caller divides by nseg).
// The clamp is one median-of-three (umax, vmax >= 0; positions are finite).
template <class GridPtr>
__device__ inline float path_sum(GridPtr G, int W, float u0, float v0, float du, float dv,
                                 int nseg, float umax, float vmax) {
  float acc = 0.f, first = 0.f, last = 0.f;
  for (int k = 0; k <= nseg; ++k) {
    const float u = __builtin_amdgcn_fmed3f(fmaf((float)k, du, u0), 0.f, umax);
    const float v = __builtin_amdgcn_fmed3f(fmaf((float)k, dv, v0), 0.f, vmax);
    const int j0 = (int)u, i0 = (int)v;
    float wx0, wx1, wx2, wx3, wz0, wz1, wz2, wz3;
    keys_weights(__builtin_amdgcn_fractf(u), wx0, wx1, wx2, wx3);  // u, v >= 0: u - j0
    keys_weights(__builtin_amdgcn_fractf(v), wz0, wz1, wz2, wz3);
    const int b = i0 * W + j0;
    const float r0 = wx0 * G[b] + wx1 * G[b + 1] + wx2 * G[b + 2] + wx3 * G[b + 3];
    const float r1 = wx0 * G[b + W] + wx1 * G[b + W + 1] + wx2 * G[b + W + 2] + wx3 * G[b + W + 3];
    const int b2 = b + 2 * W;
    const float r2 = wx0 * G[b2] + wx1 * G[b2 + 1] + wx2 * G[b2 + 2] + wx3 * G[b2 + 3];
    const float r3 = wx0 * G[b2 + W] + wx1 * G[b2 + W + 1] + wx2 * G[b2 + W + 2] + wx3 * G[b2 + W + 3];
    const float val = wz0 * r0 + wz1 * r1 + wz2 * r2 + wz3 * r3;
    acc += val;
    if (k == 0) first = val;
    if (k == nseg) last = val;
  }
  return acc - 0.5f * (first + last);
}

}  // namespace af
