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

// Layouts of the slowness deviation in LDS: the padded node grid at its own row
// stride, the same at the fixed stride TAB_LDS_W (grids with nx + 3 <= TAB_LDS_W:
// the 16 taps of a path point are then immediate offsets from one address), the
// row polynomials of the cells (ROWPOLY), or the full bicubic polynomial of every
// cell (CELLPOLY: four times the row polynomials' bytes, fewer instructions).
enum { GRID_W = 0, GRID_FIXED = 1, ROWPOLY = 2, CELLPOLY = 3 };

// Row polynomials: along a row of the padded grid, the Keys interpolation inside
// cell column j0 (nodes j0 - 1 .. j0 + 2, values g0..g3) is the cubic
// q.x + q.y f + q.z f^2 + q.w f^3 in the fraction f, with the Keys weights'
// coefficients folded into q.  Stored column-major, [j0][padded row], so the four
// rows a path point needs are 64 contiguous bytes.
__device__ __forceinline__ float4 row_poly(float g0, float g1, float g2, float g3) {
  return make_float4(g1, 0.5f * (g2 - g0), fmaf(-2.5f, g1, g0) + fmaf(2.0f, g2, -0.5f * g3),
                     1.5f * (g1 - g2) + 0.5f * (g3 - g0));
}

// path_sum over the row polynomials H ([nx][R] float4, R = nz + 3 padded rows): per
// point four rows by Horner in the x fraction, then the Keys weights in z.
__device__ __forceinline__ float path_sum_rowpoly(const float4* H, int R, float u0, float v0,
                                                  float du, float dv, int nseg, float umax,
                                                  float vmax) {
  float acc = 0.f, first = 0.f, last = 0.f;
  for (int k = 0; k <= nseg; ++k) {
    const float u = __builtin_amdgcn_fmed3f(fmaf((float)k, du, u0), 0.f, umax);
    const float v = __builtin_amdgcn_fmed3f(fmaf((float)k, dv, v0), 0.f, vmax);
    const int j0 = (int)u, i0 = (int)v;
    const float f = __builtin_amdgcn_fractf(u);  // u, v >= 0: u - j0
    float wz0, wz1, wz2, wz3;
    keys_weights(__builtin_amdgcn_fractf(v), wz0, wz1, wz2, wz3);
    const float4* q = H + j0 * R + i0;
    float r[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float4 c = q[i];
      r[i] = fmaf(fmaf(fmaf(c.w, f, c.z), f, c.y), f, c.x);
    }
    const float val = wz0 * r[0] + wz1 * r[1] + wz2 * r[2] + wz3 * r[3];
    acc += val;
    if (k == 0) first = val;
    if (k == nseg) last = val;
  }
  return acc - 0.5f * (first + last);
}

// Cell polynomials: inside cell (j0, i0) the bicubic Keys interpolant is
// sum over b of g^b P_b(f), P_b(f) = c[b].x + c[b].y f + c[b].z f^2 + c[b].w f^3 (f,
// g: the x and z fractions).  With q_r the row polynomials of the cell's padded rows
// i0 .. i0 + 3, c[b] = sum over r of K[r][b] q_r, where K[r][b] is the coefficient
// of g^b in the Keys weight of row r.  Stored as four float4 per cell, cells
// column-major ([j0][i0]), so a point reads 64 contiguous bytes.
__device__ __forceinline__ void cell_poly(const float4 (&q)[4], float4 (&c)[4]) {
  c[0] = q[1];
  c[1] = make_float4(0.5f * (q[2].x - q[0].x), 0.5f * (q[2].y - q[0].y),
                     0.5f * (q[2].z - q[0].z), 0.5f * (q[2].w - q[0].w));
#define AF_C2(k) (fmaf(-2.5f, q[1].k, q[0].k) + fmaf(2.0f, q[2].k, -0.5f * q[3].k))
#define AF_C3(k) (1.5f * (q[1].k - q[2].k) + 0.5f * (q[3].k - q[0].k))
  c[2] = make_float4(AF_C2(x), AF_C2(y), AF_C2(z), AF_C2(w));
  c[3] = make_float4(AF_C3(x), AF_C3(y), AF_C3(z), AF_C3(w));
#undef AF_C2
#undef AF_C3
}

// path_sum over the cell polynomials C ([nx][nz][4] float4): per point four
// Horner rows in the x fraction, then Horner in the z fraction.
__device__ __forceinline__ float path_sum_cellpoly(const float4* C, int nz, float u0, float v0,
                                                   float du, float dv, int nseg, float umax,
                                                   float vmax) {
  float acc = 0.f, first = 0.f, last = 0.f;
  for (int k = 0; k <= nseg; ++k) {
    const float u = __builtin_amdgcn_fmed3f(fmaf((float)k, du, u0), 0.f, umax);
    const float v = __builtin_amdgcn_fmed3f(fmaf((float)k, dv, v0), 0.f, vmax);
    const int j0 = (int)u, i0 = (int)v;
    const float f = __builtin_amdgcn_fractf(u), gz = __builtin_amdgcn_fractf(v);  // u, v >= 0
    const float4* q = C + 4 * (j0 * nz + i0);
    float r[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const float4 c = q[b];
      r[b] = fmaf(fmaf(fmaf(c.w, f, c.z), f, c.y), f, c.x);
    }
    const float val = fmaf(fmaf(fmaf(r[3], gz, r[2]), gz, r[1]), gz, r[0]);
    acc += val;
    if (k == 0) first = val;
    if (k == nseg) last = val;
  }
  return acc - 0.5f * (first + last);
}

// One instantiation per refraction mode (arc or flat lens, root or discrete
// search), so the default mode keeps its own register allocation, and per layout.
// A workgroup of ITEMS x 256 threads takes ITEMS consecutive work items (one point
// per thread) over one LDS copy: where only two polynomial copies fit a CU, three
// items per copy keep 6 waves per SIMD (within the kernel's 80 registers).
template <int MODE, int LAYOUT, int ITEMS>
__global__ __launch_bounds__(256 * ITEMS) __attribute__((amdgpu_waves_per_eu(6)))
void k_table(TableArgs A) {
  extern __shared__ float G[];
  const Geo& g = A.g;
  const int WL = LAYOUT == GRID_FIXED ? TAB_LDS_W : g.W;
  const int RP = g.nz + 3;
  if (LAYOUT == CELLPOLY) {
    float4* H = reinterpret_cast<float4*>(G);
    for (int i = threadIdx.x; i < g.nx * g.nz; i += 256 * ITEMS) {
      const int j0 = i / g.nz, i0 = i - j0 * g.nz;
      float4 q[4], c[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float* row = A.gdev + (i0 + r) * g.W + j0;
        q[r] = row_poly(row[0], row[1], row[2], row[3]);
      }
      cell_poly(q, c);
#pragma unroll
      for (int b = 0; b < 4; ++b) H[4 * i + b] = c[b];
    }
  } else if (LAYOUT == ROWPOLY) {
    float4* H = reinterpret_cast<float4*>(G);
    for (int i = threadIdx.x; i < g.nx * RP; i += 256 * ITEMS) {
      const int j0 = i / RP, r = i - j0 * RP;
      const float* row = A.gdev + r * g.W + j0;
      H[i] = row_poly(row[0], row[1], row[2], row[3]);
    }
  } else {
    for (int i = threadIdx.x; i < WL * RP; i += 256 * ITEMS) {
      const int r = i / WL, c = i - r * WL;
      G[i] = c < g.W ? A.gdev[r * g.W + c] : 0.f;
    }
  }
  __syncthreads();
  const int item = blockIdx.x * ITEMS + (int)(threadIdx.x >> 8);
  if (item >= A.n_work) return;  // the last workgroup's second item (no barrier follows)
  const int2 w = A.work[item];
  const int tile = w.x, a0 = w.y;
  const int4 tr = A.tiles[tile];

  const long long p = (long long)tile * TILE + (threadIdx.x & 255);
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
        const float acc =
            LAYOUT == CELLPOLY
                ? path_sum_cellpoly(reinterpret_cast<const float4*>(G), g.nz, u0, v0,
                                    (up - u0) * inv_n, (vp - v0) * inv_n, g.n_seg, umax, vmax)
            : LAYOUT == ROWPOLY
                ? path_sum_rowpoly(reinterpret_cast<const float4*>(G), RP, u0, v0,
                                   (up - u0) * inv_n, (vp - v0) * inv_n, g.n_seg, umax, vmax)
                : path_sum(G, WL, u0, v0, (up - u0) * inv_n, (vp - v0) * inv_n, g.n_seg, umax,
                           vmax);
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
  A.n_work = c->v.n_tab_work;
  A.gdev = c->d_gdev.as<float>();
  A.scal = c->d_scal.as<double>();
  A.tab = c->d_tab.as<TabEntry>();
  A.ray_uv = c->d_ray_uv.as<float2>();
  A.ray_l2 = c->d_ray_l2.as<float>();
  if (c->v.n_tab_work == 0) return hipSuccess;
  // The cell polynomials, then the row polynomials, where six 256-thread
  // workgroups fit a CU's LDS, or two of 512 threads; else the padded grid at the
  // fixed row stride where its copy fits the LDS of a workgroup, else at the grid's
  // own.
  const size_t cellp = 4 * sizeof(float4) * (size_t)c->nx * c->nz;
  const size_t poly = sizeof(float4) * (size_t)c->nx * (c->nz + 3);
  const bool fixed = c->nx + 3 <= TAB_LDS_W &&
                     sizeof(float) * (size_t)TAB_LDS_W * (c->nz + 3) <= TAB_LDS_BYTES;
  const int layout = cellp * 2 <= TAB_LDS_BYTES  ? CELLPOLY
                     : poly * 2 <= TAB_LDS_BYTES ? ROWPOLY
                     : fixed                     ? GRID_FIXED
                                                 : GRID_W;
  const size_t bytes = layout == CELLPOLY ? cellp : poly;
  // (two copies per CU: three items per copy, 6 waves per SIMD)
  const int items = (layout == CELLPOLY || layout == ROWPOLY) && bytes * 6 > TAB_LDS_BYTES ? 3 : 1;
  const size_t lds = layout == CELLPOLY || layout == ROWPOLY
                         ? bytes
                         : sizeof(float) * (size_t)(fixed ? TAB_LDS_W : c->nx + 3) * (c->nz + 3);
  const dim3 grid((c->v.n_tab_work + items - 1) / items), block(256 * items);
#define AF_TABLE_LAUNCH(M)                                                          \
  if (layout == CELLPOLY && items == 3)                                             \
    hipLaunchKernelGGL((k_table<M, CELLPOLY, 3>), grid, block, lds, c->stream, A); \
  else if (layout == CELLPOLY)                                                      \
    hipLaunchKernelGGL((k_table<M, CELLPOLY, 1>), grid, block, lds, c->stream, A); \
  else if (layout == ROWPOLY && items == 3)                                         \
    hipLaunchKernelGGL((k_table<M, ROWPOLY, 3>), grid, block, lds, c->stream, A);  \
  else if (layout == ROWPOLY)                                                       \
    hipLaunchKernelGGL((k_table<M, ROWPOLY, 1>), grid, block, lds, c->stream, A);  \
  else if (layout == GRID_FIXED)                                                    \
    hipLaunchKernelGGL((k_table<M, GRID_FIXED, 1>), grid, block, lds, c->stream, A); \
  else                                                                              \
    hipLaunchKernelGGL((k_table<M, GRID_W, 1>), grid, block, lds, c->stream, A);
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
