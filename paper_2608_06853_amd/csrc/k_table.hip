// Travel-time table: for every active (element, point) pair, the bent-ray time
// T = L1/c_lens + L2 * (trapezoid sum of bicubic slowness)/N (Eqs. 1, 7-8 and
// Section III-A), stored as the sample position and apodised phasor DAS needs.
//
// FP64 appears only inside the lens refraction (trace_lens): the homogeneous
// time T_hom = L1/c_lens + L2/c_med at the stationary point.  The path integral
// is taken over the deviation s - s_med in FP32, so T = T_hom + dT with dT small;
// the sample index and the phase are reduced from T_hom in FP64 before dT is
// added in FP32.
#include "af_internal.h"

namespace af {
namespace {

// Row stride of the LDS grid copy for grids up to 64 nodes wide: as a constant,
// the 16 taps of a path point are immediate offsets from one LDS address.
constexpr int TAB_LDS_W = 67;
constexpr size_t TAB_LDS_BYTES = 160 * 1024;  // LDS of one workgroup on gfx950

// One instantiation per refraction mode (arc or flat lens, root or discrete
// search), so the default mode keeps its own register allocation; FIXED_W copies
// the grid at row stride TAB_LDS_W (grids with nx + 3 <= TAB_LDS_W).
template <int MODE, bool FIXED_W>
__global__ __launch_bounds__(256) void k_table(TableArgs A) {
  extern __shared__ float G[];
  const Geo& g = A.g;
  const int2 w = A.work[blockIdx.x];
  const int tile = w.x, a0 = w.y;
  const int4 tr = A.tiles[tile];
  const int WL = FIXED_W ? TAB_LDS_W : g.W;
  const int gsz = WL * (g.nz + 3);
  for (int i = threadIdx.x; i < gsz; i += 256) {
    const int r = i / WL, c = i - r * WL;
    G[i] = c < g.W ? A.gdev[r * g.W + c] : 0.f;
  }
  __syncthreads();

  const long long p = (long long)tile * TILE + threadIdx.x;
  const int2 pr = A.prange[p];
  const double4 pp = A.ptpol[p];
  const float2 pxy = A.ptxy[p];
  const double icm = A.scal[1];
  const float inv_n = 1.f / (float)g.n_seg;
  const float up = (pxy.x - g.x0) * g.idx, vp = (pxy.y - g.z0) * g.idz;
  const float umax = (float)(g.nx - 1), vmax = (float)(g.nz - 1);
  const double half_ttp = 0.5 * g.t_ttp;
  const double u_off = half_ttp - 0.5 * g.t0;
  const float fsf = (float)g.fs, fdf = (float)g.fd;
  const int a1 = min(a0 + TAB_CHUNK - 1, tr.y);
  for (int a = a0; a <= a1; ++a) {
    TabEntry e;
    float2 ruv = make_float2(0.f, 0.f);
    float rl2 = 0.f;
    if (a < pr.x || a > pr.y) {
      e.ui = 0;  // masked: zero phasor (and a sample index inside every record)
      e.uf = 0.f;
      e.er = 0.f;
      e.ei = 0.f;
    } else {
      const double4 el = A.elem[a];
      const RayOut r = refract<MODE>(el, pp, g.dlens, g.icl, icm, g.nsearch);
      const float u0 = (r.refx - g.x0) * g.idx, v0 = (r.refz - g.z0) * g.idz;
      // A slowness that is not finite and positive (reported by af_set_slowness; a
      // caller's own s in the optimiser loop is not re-read on the host) can give a
      // non-finite ray or time.  Such an entry is written as masked, so every sample
      // index the DAS kernels form stays bounded (|ui| < 2^29) and every grid
      // position the path kernels clamp is finite.
      bool ok = isfinite(u0) && isfinite(v0) && isfinite(r.l2) && isfinite(r.t_hom);
      float dT = 0.f;
      double uh = 0.0;
      if (ok) {
        const float acc = path_sum(G, WL, u0, v0, (up - u0) * inv_n, (vp - v0) * inv_n,
                                   g.n_seg, umax, vmax);
        dT = r.l2 * acc * inv_n;
        uh = (r.t_hom + u_off) * g.fs;
        ok = fabs(uh) < 268435456.0 && fabsf(dT * fsf) < 268435456.f;  // 2^28; false for NaN
      }
      if (ok) {
        ruv = make_float2(u0, v0);
        rl2 = r.l2;
        const double kh = floor(uh);
        float uf = (float)(uh - kh) + dT * fsf;
        const float cf = floorf(uf);
        e.ui = (int)kh + (int)cf;
        e.uf = uf - cf;
        double cyc = (r.t_hom + half_ttp) * g.fd;
        cyc -= rint(cyc);
        const float cy = (float)cyc + dT * fdf;
        float sn, cs;
        sincospif(2.f * cy, &sn, &cs);
        e.er = cs;
        e.ei = sn;
      } else {
        e.ui = 0;
        e.uf = 0.f;
        e.er = 0.f;
        e.ei = 0.f;
      }
    }
    A.tab[(size_t)a * g.P + p] = e;
    A.ray_uv[(size_t)a * g.P + p] = ruv;
    A.ray_l2[(size_t)a * g.P + p] = rl2;
  }
}

}  // namespace

hipError_t launch_table(af_ctx* c) {
  TableArgs A;
  A.g = c->geo();
  A.elem = c->d_elem.as<double4>();
  A.ptpol = c->v.ptpol;
  A.ptxy = c->v.ptxy;
  A.prange = c->v.prange;
  A.tiles = c->v.tiles;
  A.work = c->v.tabwork;
  A.gdev = c->d_gdev.as<float>();
  A.scal = c->d_scal.as<double>();
  A.tab = c->d_tab.as<TabEntry>();
  A.ray_uv = c->d_ray_uv.as<float2>();
  A.ray_l2 = c->d_ray_l2.as<float>();
  if (c->v.n_tab_work == 0) return hipSuccess;
  // the fixed row stride only where its copy fits the LDS of a workgroup
  const bool fixed = c->nx + 3 <= TAB_LDS_W &&
                     sizeof(float) * (size_t)TAB_LDS_W * (c->nz + 3) <= TAB_LDS_BYTES;
  const size_t lds = sizeof(float) * (size_t)(fixed ? TAB_LDS_W : c->nx + 3) * (c->nz + 3);
  const dim3 grid(c->v.n_tab_work), block(256);
#define AF_TABLE_LAUNCH(M)                                                        \
  if (fixed)                                                                      \
    hipLaunchKernelGGL((k_table<M, true>), grid, block, lds, c->stream, A);      \
  else                                                                            \
    hipLaunchKernelGGL((k_table<M, false>), grid, block, lds, c->stream, A);
  switch (refract_mode(A.g.flat != 0, A.g.nsearch, A.g.dlens)) {
    case ARC_ROOT: AF_TABLE_LAUNCH(ARC_ROOT); break;
    case ARC_SEARCH: AF_TABLE_LAUNCH(ARC_SEARCH); break;
    case FLAT_ROOT: AF_TABLE_LAUNCH(FLAT_ROOT); break;
    default: AF_TABLE_LAUNCH(FLAT_SEARCH);
  }
#undef AF_TABLE_LAUNCH
  return hipGetLastError();
}

}  // namespace af
