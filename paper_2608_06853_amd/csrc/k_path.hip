// Adjoint of the path integral: dL/ds[node] += sum over rays and ray points of
// dL/dT * L2 * w_k * (bicubic weight of the node at r_k) / N.  Refraction points
// and c_med are held constant (they follow the global mean speed).
//
// A workgroup takes one tile of points and every active element of it.  The
// rays of a wavefront are nearly parallel, so at a given k their lanes touch the
// same grid nodes; the workgroup therefore scatters into `copies` interleaved
// private copies of the padded grid in LDS (copy = lane mod copies) so lanes
// that hit one node land in different banks.  The copies are summed at the end
// and added to the global padded grid with one atomic per node.
#include "af_internal.h"

namespace af {
namespace {

__global__ __launch_bounds__(256) void k_path_adj(PathArgs A) {
  extern __shared__ float sg[];
  const Geo& g = A.g;
  const int tid = threadIdx.x;
  const int tile = A.order[blockIdx.x];
  const int4 tr = A.tiles[tile];
  const int C = A.copies;
  const int W = g.W;
  const int nodes = W * (g.nz + 3);
  for (int i = tid; i < nodes * C; i += 256) sg[i] = 0.f;
  __syncthreads();

  const long long p = (long long)tile * TILE + tid;
  const int2 pr = A.prange[p];
  const double4 pp = A.ptpol[p];
  const float2 pxy = A.ptxy[p];
  const double icm = A.scal[1];
  const float inv_n = 1.f / (float)g.n_seg;
  const float up = (pxy.x - g.x0) * g.idx, vp = (pxy.y - g.z0) * g.idz;
  const float umax = (float)(g.nx - 1), vmax = (float)(g.nz - 1);
  const int lc = tid % C;
  const int a_lo = max(tr.x, pr.x), a_hi = min(tr.y, pr.y);
  for (int a = a_lo; a <= a_hi; ++a) {
    const float gbar = A.gT[(long long)a * g.P + p];
    if (gbar == 0.f) continue;
    const double4 el = A.elem[a];
    const RayOut r = trace_lens(el.x, el.y, el.z, pp.x, pp.y, pp.z, g.dlens, g.icl, icm);
    const float coef = gbar * r.l2 * inv_n;
    const float u0 = (r.refx - g.x0) * g.idx, v0 = (r.refz - g.z0) * g.idz;
    const float du = (up - u0) * inv_n, dv = (vp - v0) * inv_n;
    for (int k = 0; k <= g.n_seg; ++k) {
      const float u = fminf(fmaxf(fmaf((float)k, du, u0), 0.f), umax);
      const float v = fminf(fmaxf(fmaf((float)k, dv, v0), 0.f), vmax);
      const int j0 = (int)u, i0 = (int)v;
      float wx[4], wz[4];
      keys_weights(u - (float)j0, wx[0], wx[1], wx[2], wx[3]);
      keys_weights(v - (float)i0, wz[0], wz[1], wz[2], wz[3]);
      const float ck = (k == 0 || k == g.n_seg) ? 0.5f * coef : coef;
      float* base = sg + (i0 * W + j0) * C + lc;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const float cr = ck * wz[rr];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) atomicAdd(base + (rr * W + cc) * C, cr * wx[cc]);
      }
    }
  }
  __syncthreads();
  for (int n = tid; n < nodes; n += 256) {
    float s = 0.f;
    for (int cc = 0; cc < C; ++cc) s += sg[n * C + cc];
    if (s != 0.f) atomicAdd(A.gpad + n, s);
  }
}

__global__ __launch_bounds__(256) void k_zero(float* __restrict__ x, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = 0.f;
}

}  // namespace

hipError_t launch_path_adj(af_ctx* c) {
  const int nodes = (c->nx + 3) * (c->nz + 3);
  hipLaunchKernelGGL(k_zero, dim3((nodes + 255) / 256), dim3(256), 0, c->stream,
                     c->d_gpad.as<float>(), (long long)nodes);
  if (c->n_order == 0) return hipGetLastError();
  int copies = 16;
  while (copies > 1 && (size_t)nodes * copies * sizeof(float) > 80 * 1024) copies >>= 1;
  PathArgs A{};
  A.g = c->geo();
  A.elem = c->d_elem.as<double4>();
  A.ptpol = c->d_ptpol.as<double4>();
  A.ptxy = c->d_ptxy.as<float2>();
  A.prange = c->d_prange.as<int2>();
  A.tiles = c->d_tiles.as<int4>();
  A.order = c->d_order.as<int>();
  A.gT = c->d_gT.as<float>();
  A.scal = c->d_scal.as<double>();
  A.gpad = c->d_gpad.as<float>();
  A.copies = copies;
  const size_t lds = sizeof(float) * (size_t)nodes * copies;
  hipLaunchKernelGGL(k_path_adj, dim3(c->n_order), dim3(256), lds, c->stream, A);
  return hipGetLastError();
}

}  // namespace af
