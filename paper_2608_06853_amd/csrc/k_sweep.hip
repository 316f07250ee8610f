// Dynamic CMPE grid (Sound Speed Estimation subsection): the evaluation points of
// the global-speed sweep at speed c_g.  Every pixel's depth below the lens surface
// is stretched by k = c_g / c_ref -- along its polar angle for a curvilinear array
// (concentric lens), straight down for a linear one (flat lens) -- and the patch
// spacing becomes lambda_g / 2 = c_g / (2 f_c), so that the same time samples are
// observed at every speed.  The pixel-to-tile assignment of the base layout is
// kept; each point's active element range (Eqs. 2 and 4, every element tested) and
// each tile's range are formed here, on the device.
#include <climits>

#include "af_internal.h"

namespace af {
namespace {

struct SweepArgs {
  int n_elem, flat;
  double k;          // c_g / c_ref
  double spacing;    // patch spacing at c_g
  double rl;         // lens surface: radius of the arc, or z of the plane
  double half_f;     // F / 2 of the apodisation |x'| <= (F / 2) z'
  const double4* base;    // per internal point: pixel centre (x, z) of the base layout and
                          // the patch offset (in units of the spacing)
  const int* i2c;         // caller point of every internal point (-1: padding)
  const double4* elemf;   // element (x, z, cos theta, sin theta), theta of Eq. 3
  double4* ptpol;         // outputs, as the geometry set-up lays them out
  float2* ptxy;
  int2* prange;
  TileStat* tstat;        // per tile: element range, active pairs and samples
};

// One workgroup per tile of 256 points.
__global__ __launch_bounds__(256) void k_sweep_points(SweepArgs A) {
  __shared__ int s_lo[256], s_hi[256], s_bad[256];
  __shared__ long long s_pairs[256], s_samples[256];
  const int tid = threadIdx.x, tile = blockIdx.x;
  const long long p = (long long)tile * TILE + tid;
  const double4 b = A.base[p];
  double x, z;
  if (A.flat) {
    x = b.x;
    z = A.rl + (b.y - A.rl) * A.k;
  } else {
    const double rho = sqrt(b.x * b.x + b.y * b.y);
    const double f = (A.rl + (rho - A.rl) * A.k) / rho;
    x = b.x * f;
    z = b.y * f;
  }
  x += b.z * A.spacing;
  z += b.w * A.spacing;
  const double r = sqrt(x * x + z * z);
  A.ptpol[p] = A.flat ? make_double4(x, z, 0.0, 0.0) : make_double4(r, x / r, z / r, 0.0);
  A.ptxy[p] = make_float2((float)x, (float)z);

  int lo = 1, hi = 0, bad = 0;
  if (A.i2c[p] >= 0) {
    int l = A.n_elem, h = -1, cnt = 0;
    for (int a = 0; a < A.n_elem; ++a) {
      const double4 e = A.elemf[a];
      const double dx = x - e.x, dz = z - e.y;
      const double xp = e.z * dx - e.w * dz;
      const double zp = e.w * dx + e.z * dz;
      if (fabs(xp) <= A.half_f * zp) {
        l = min(l, a);
        h = max(h, a);
        ++cnt;
      }
    }
    if (cnt > 0) {
      lo = l;
      hi = h;
      bad = cnt != h - l + 1;  // the active elements of a point must be contiguous
    }
  }
  A.prange[p] = make_int2(lo, hi);

  const long long n = lo <= hi ? hi - lo + 1 : 0;
  s_lo[tid] = lo <= hi ? lo : INT_MAX;
  s_hi[tid] = lo <= hi ? hi : -1;
  s_bad[tid] = bad;
  s_pairs[tid] = n;
  s_samples[tid] = n * n;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      s_lo[tid] = min(s_lo[tid], s_lo[tid + st]);
      s_hi[tid] = max(s_hi[tid], s_hi[tid + st]);
      s_bad[tid] |= s_bad[tid + st];
      s_pairs[tid] += s_pairs[tid + st];
      s_samples[tid] += s_samples[tid + st];
    }
    __syncthreads();
  }
  if (tid == 0) {
    TileStat ts;
    ts.lo = s_hi[0] >= 0 ? s_lo[0] : A.n_elem;
    ts.hi = s_hi[0];
    ts.bad = s_bad[0];
    ts.pairs = s_pairs[0];
    ts.samples = s_samples[0];
    A.tstat[tile] = ts;
  }
}

}  // namespace

hipError_t launch_sweep_points(af_ctx* c, double k, double spacing, double rl, TileStat* tstat) {
  SweepArgs A;
  A.n_elem = c->N;
  A.flat = c->flat ? 1 : 0;
  A.k = k;
  A.spacing = spacing;
  A.rl = rl;
  A.half_f = 0.5 * c->fnum;
  A.base = c->d_dyn_base.as<double4>();
  A.i2c = c->d_i2c.as<int>();
  A.elemf = c->d_elemf.as<double4>();
  A.ptpol = c->d_ptpol.as<double4>();
  A.ptxy = c->d_ptxy.as<float2>();
  A.prange = c->d_prange.as<int2>();
  A.tstat = tstat;
  hipLaunchKernelGGL(k_sweep_points, dim3(c->n_tiles), dim3(256), 0, c->stream, A);
  return hipGetLastError();
}

}  // namespace af
