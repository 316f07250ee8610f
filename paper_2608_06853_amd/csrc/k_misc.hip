// Small kernels around the hot path: global mean speed and the padded deviation
// grid, deadzone regularisers (Eqs. 10-11) with their gradient, the loss terms
// (Eq. 12), the final scaling of the block-image gradient, the fold of the
// padded grid gradient onto the nodes, and the Adam update.
#include "af_internal.h"

namespace af {
namespace {

struct RegP {
  float w1, kx1, kz1, w2, kx2, kz2;
  double dx, dz;
};

__device__ inline double dz_grad(double x, double k) { return fabs(x) > k ? (x > 0 ? 1.0 : -1.0) : 0.0; }
__device__ inline double dz_val(double x, double k) { return fmax(0.0, fabs(x) - k); }

__device__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// scal: [0] c_med, [1] s_med = 1/c_med, [2] non-finite flag, [3] R_TV, [4] R_SV,
//       [5] 1/n_valid, [6] n_valid
__global__ __launch_bounds__(256) void k_prepare_grid(const float* __restrict__ s, int nx, int nz,
                                                      float* __restrict__ gdev, double* scal,
                                                      int do_reg, RegP rp, float* __restrict__ regg) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int n = nx * nz;
  double acc = 0.0, bad = 0.0;
  for (int i = t; i < n; i += 256) {
    const float v = s[i];
    if (!(v > 0.f) || !isfinite(v)) bad = 1.0;
    acc += 1.0 / (double)v;
  }
  const double sum = block_sum(acc, red);
  const double nbad = block_sum(bad, red);
  const double c_med = sum / n;
  const double s_med = 1.0 / c_med;
  if (t == 0) {
    scal[0] = c_med;
    scal[1] = s_med;
    scal[2] = nbad;
  }
  const int W = nx + 3, H = nz + 3;
  for (int idx = t; idx < W * H; idx += 256) {
    const int pi = idx / W, pj = idx - pi * W;
    const int i = min(max(pi - 1, 0), nz - 1), j = min(max(pj - 1, 0), nx - 1);
    gdev[idx] = (float)((double)s[i * nx + j] - s_med);
  }
  if (!do_reg) return;
  auto C = [&](int i, int j) { return 1.0 / (double)s[i * nx + j]; };
  const double idx1 = 1.0 / rp.dx, idz1 = 1.0 / rp.dz;
  const double idx2 = idx1 * idx1, idz2 = idz1 * idz1;
  double tv = 0.0, sv = 0.0;
  for (int idx = t; idx < n; idx += 256) {
    const int i = idx / nx, j = idx - i * nx;
    const double c = C(i, j);
    // stencils owned by this node
    if (j < nx - 1) tv += dz_val((C(i, j + 1) - c) * idx1, rp.kx1);
    if (i < nz - 1) tv += dz_val((C(i + 1, j) - c) * idz1, rp.kz1);
    if (j >= 1 && j <= nx - 2) sv += dz_val((C(i, j + 1) - 2.0 * c + C(i, j - 1)) * idx2, rp.kx2);
    if (i >= 1 && i <= nz - 2) sv += dz_val((C(i + 1, j) - 2.0 * c + C(i - 1, j)) * idz2, rp.kz2);
    // gradient by gathering every stencil that touches this node
    double g1 = 0.0, g2 = 0.0;
    if (j >= 1) g1 += dz_grad((c - C(i, j - 1)) * idx1, rp.kx1) * idx1;
    if (j <= nx - 2) g1 -= dz_grad((C(i, j + 1) - c) * idx1, rp.kx1) * idx1;
    if (i >= 1) g1 += dz_grad((c - C(i - 1, j)) * idz1, rp.kz1) * idz1;
    if (i <= nz - 2) g1 -= dz_grad((C(i + 1, j) - c) * idz1, rp.kz1) * idz1;
    auto sxx = [&](int jj) { return (C(i, jj + 1) - 2.0 * C(i, jj) + C(i, jj - 1)) * idx2; };
    auto szz = [&](int ii) { return (C(ii + 1, j) - 2.0 * C(ii, j) + C(ii - 1, j)) * idz2; };
    if (j - 1 >= 1 && j - 1 <= nx - 2) g2 += dz_grad(sxx(j - 1), rp.kx2) * idx2;
    if (j >= 1 && j <= nx - 2) g2 -= 2.0 * dz_grad(sxx(j), rp.kx2) * idx2;
    if (j + 1 >= 1 && j + 1 <= nx - 2) g2 += dz_grad(sxx(j + 1), rp.kx2) * idx2;
    if (i - 1 >= 1 && i - 1 <= nz - 2) g2 += dz_grad(szz(i - 1), rp.kz2) * idz2;
    if (i >= 1 && i <= nz - 2) g2 -= 2.0 * dz_grad(szz(i), rp.kz2) * idz2;
    if (i + 1 >= 1 && i + 1 <= nz - 2) g2 += dz_grad(szz(i + 1), rp.kz2) * idz2;
    const double gc = ((double)rp.w1 * g1 + (double)rp.w2 * g2) / n;
    regg[idx] = (float)(-gc * c * c);
  }
  const double tvs = block_sum(tv, red);
  const double svs = block_sum(sv, red);
  if (t == 0) {
    scal[3] = tvs / n;
    scal[4] = svs / n;
  }
}

// Fixed-order reduction of the CMPE partials into the loss terms.
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ part, int n_part,
                                                  double* scal, float* __restrict__ terms,
                                                  af_loss_params lp, int n_pix) {
  __shared__ double red[256];
  double e = 0, nv = 0, b = 0;
#pragma unroll 4
  for (int i = threadIdx.x; i < n_part; i += 256) {  // unrolled: loads of 4 partials in flight
    e += part[4 * i + 0];
    nv += part[4 * i + 1];
    b += part[4 * i + 2];
  }
  e = block_sum(e, red);
  nv = block_sum(nv, red);
  b = block_sum(b, red);
  if (threadIdx.x == 0) {
    const double cmpe = nv > 0 ? e / nv : 0.0;
    const double sb = b / n_pix / (double)lp.sb_ref;
    const double tv = scal[3], sv = scal[4];
    double total = cmpe + (double)lp.w1 * tv + (double)lp.w2 * sv - (double)lp.w_sb * sb;
    if (scal[2] != 0.0) total = __longlong_as_double(0x7ff8000000000000ULL);
    scal[5] = nv > 0 ? 1.0 / nv : 0.0;
    scal[6] = nv;
    terms[AF_TERM_CMPE] = (float)cmpe;
    terms[AF_TERM_TV] = (float)tv;
    terms[AF_TERM_SV] = (float)sv;
    terms[AF_TERM_SB] = (float)sb;
    terms[AF_TERM_TOTAL] = (float)total;
    terms[AF_TERM_NVALID] = (float)nv;
    terms[AF_TERM_CMED] = (float)scal[0];
    terms[7] = 0.f;
  }
}

// G <- G / n_valid + dSB/dB (centre points) over the active blocks of every sub-tile.
__global__ __launch_bounds__(64) void k_gscale(Geo g, const int4* __restrict__ tiles,
                                               float2* __restrict__ gblk,
                                               const float2* __restrict__ gsb,
                                               const double* __restrict__ scal) {
  const long long p = (long long)blockIdx.x * SUB + threadIdx.x;
  const int4 tr = tiles[p / TILE];
  if (tr.x > tr.y) return;
  const float inv = (float)scal[5];
  const float2 sb = gsb[p];
  for (int i = tr.z; i <= tr.w; ++i)
    for (int j = tr.z; j <= tr.w; ++j) {
      const long long o = ((long long)i * g.nblk + j) * g.P + p;
      float2 v = gblk[o];
      v.x = fmaf(v.x, inv, sb.x);
      v.y = fmaf(v.y, inv, sb.y);
      gblk[o] = v;
    }
}

// Sum the padded-grid gradient onto the clamped nodes and add the regulariser.
__global__ __launch_bounds__(256) void k_grad_fold(const float* __restrict__ gpad,
                                                   const float* __restrict__ regg, int nx, int nz,
                                                   float* __restrict__ grad) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nx * nz) return;
  const int i = idx / nx, j = idx - i * nx;
  const int W = nx + 3;
  const int pi0 = (i == 0) ? 0 : i + 1, pi1 = (i == nz - 1) ? nz + 2 : i + 1;
  const int pj0 = (j == 0) ? 0 : j + 1, pj1 = (j == nx - 1) ? nx + 2 : j + 1;
  float acc = regg ? regg[idx] : 0.f;
  for (int pi = pi0; pi <= pi1; ++pi)
    for (int pj = pj0; pj <= pj1; ++pj) acc += gpad[pi * W + pj];
  grad[idx] = acc;
}

__global__ __launch_bounds__(256) void k_adam(int n, float lr, float b1, float b2, float eps,
                                              float bc1, float bc2, float* __restrict__ s,
                                              float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ grad,
                                              float* __restrict__ s_copy) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float si = s[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  s[i] = si;
  s_copy[i] = si;
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ x, int n, float v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = v;
}

}  // namespace

hipError_t launch_fill(af_ctx* c, float* x, int n, float v) {
  hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, c->stream, x, n, v);
  return hipGetLastError();
}

hipError_t launch_prepare_grid(af_ctx* c, const float* s, int nx, int nz, float* gdev, double* scal,
                               int do_reg, const af_loss_params* lp, float* regg) {
  RegP rp{};
  if (lp) rp = RegP{lp->w1, lp->kx1, lp->kz1, lp->w2, lp->kx2, lp->kz2, c->dx, c->dz};
  hipLaunchKernelGGL(k_prepare_grid, dim3(1), dim3(256), 0, c->stream, s, nx, nz, gdev, scal,
                     do_reg, rp, regg);
  return hipGetLastError();
}

hipError_t launch_finalize(af_ctx* c, const af_loss_params* lp, float* terms) {
  const int n_part = (int)(c->P_int / SUB);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, c->stream, c->d_part.as<double>(), n_part,
                     c->d_scal.as<double>(), terms, *lp, c->n_pix);
  return hipGetLastError();
}

hipError_t launch_gscale(af_ctx* c, float2* gblk) {
  hipLaunchKernelGGL(k_gscale, dim3((unsigned)(c->P_int / SUB)), dim3(64), 0, c->stream, c->geo(),
                     c->d_tiles.as<int4>(), gblk, c->d_gsb.as<float2>(), c->d_scal.as<double>());
  return hipGetLastError();
}

hipError_t launch_grad_fold(af_ctx* c, float* grad) {
  const int n = c->nx * c->nz;
  hipLaunchKernelGGL(k_grad_fold, dim3((n + 255) / 256), dim3(256), 0, c->stream,
                     c->d_gpad.as<float>(), c->d_regg.as<float>(), c->nx, c->nz, grad);
  return hipGetLastError();
}

hipError_t launch_adam(af_ctx* c, const af_adam_params* ap, int step, float* s, float* m, float* v,
                       const float* grad) {
  const int n = c->nx * c->nz;
  const float bc1 = 1.f - powf(ap->beta1, (float)step);
  const float bc2 = 1.f - powf(ap->beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, ap->lr, ap->beta1,
                     ap->beta2, ap->eps, bc1, bc2, s, m, v, grad, c->d_s.as<float>());
  return hipGetLastError();
}

}  // namespace af
