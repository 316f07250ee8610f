// Channel-data simulator for synthetic workloads: point scatterers echo a
// baseband Gaussian envelope at their bent-ray round-trip time through a true
// slowness map (same ray model as the beamformer), with the demodulation phase
// exp(-j 2 pi fd tau).  One workgroup builds one (transmit, receive) record in
// LDS and writes it once.
#include "af_internal.h"

namespace af {
namespace {

struct SimGeo {
  int nx, nz, W, n_seg;
  float x0, z0, idx, idz;
};

__global__ __launch_bounds__(256) void k_sim_times(Geo g, SimGeo sgeo, const double4* __restrict__ elem,
                                                   const double4* __restrict__ spol,
                                                   const float2* __restrict__ sxy, int n_scat,
                                                   const float* __restrict__ gdev,
                                                   const double* __restrict__ scal,
                                                   double* __restrict__ T) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  const int a = blockIdx.y;
  if (k >= n_scat) return;
  const double4 el = elem[a];
  const double4 pp = spol[k];
  const RayOut r = g.flat ? trace_flat(el.x, el.y, pp.x, pp.y, g.dlens, g.icl, scal[1], 0)
                         : trace_lens(el.x, el.y, el.z, pp.x, pp.y, pp.z, g.dlens, g.icl, scal[1]);
  const float inv_n = 1.f / (float)sgeo.n_seg;
  const float u0 = (r.refx - sgeo.x0) * sgeo.idx, v0 = (r.refz - sgeo.z0) * sgeo.idz;
  const float up = (sxy[k].x - sgeo.x0) * sgeo.idx, vp = (sxy[k].y - sgeo.z0) * sgeo.idz;
  const float acc = path_sum(gdev, sgeo.W, u0, v0, (up - u0) * inv_n, (vp - v0) * inv_n,
                             sgeo.n_seg, (float)(sgeo.nx - 1), (float)(sgeo.nz - 1));
  T[(long long)a * n_scat + k] = r.t_hom + (double)(r.l2 * acc * inv_n);
}

// The echoes of all scatterers are summed into the record in 64-bit fixed point
// (units of 2^-32): integer adds commute, so the record is the same on every run
// whatever order the threads' atomic adds land in (float adds would round
// differently), and the simulated channel data repeat bit for bit.
constexpr double SIM_FIX = 4294967296.0;  // 2^32

__device__ inline unsigned long long sim_fixed(float v) {
  return (unsigned long long)__double2ll_rn((double)v * SIM_FIX);  // |v| < 2^31
}

__global__ __launch_bounds__(256) void k_sim_synth(Geo g, const double* __restrict__ T, int n_scat,
                                                   const float* __restrict__ amp, double sigma,
                                                   float2* __restrict__ iq) {
  extern __shared__ unsigned long long rec[];  // [2 * ns], fixed point
  const int t = blockIdx.x / g.n_elem, r = blockIdx.x % g.n_elem;
  const int ns = g.ns;
  for (int i = threadIdx.x; i < 2 * ns; i += 256) rec[i] = 0ull;
  __syncthreads();
  const double half = 6.0 * sigma;
  const float inv2s2 = (float)(0.5 / (sigma * sigma));
  for (int k = threadIdx.x; k < n_scat; k += 256) {
    const double tau = T[(long long)t * n_scat + k] + T[(long long)r * n_scat + k] + g.t_ttp;
    int n0 = (int)ceil((tau - half - g.t0) * g.fs);
    int n1 = (int)floor((tau + half - g.t0) * g.fs);
    n0 = max(n0, 0);
    n1 = min(n1, ns - 1);
    if (n0 > n1) continue;
    double cyc = g.fd * tau;
    cyc -= rint(cyc);
    float sn, cs;
    sincospif(-2.f * (float)cyc, &sn, &cs);
    const float a = amp[k];
    const float px = a * cs, py = a * sn;
    for (int n = n0; n <= n1; ++n) {
      const float dt = (float)(g.t0 + n / g.fs - tau);
      const float e = __expf(-dt * dt * inv2s2);
      atomicAdd(&rec[2 * n], sim_fixed(e * px));
      atomicAdd(&rec[2 * n + 1], sim_fixed(e * py));
    }
  }
  __syncthreads();
  float2* out = iq + ((long long)t * g.n_elem + r) * ns;
  for (int i = threadIdx.x; i < ns; i += 256)
    out[i] = make_float2((float)((double)(long long)rec[2 * i] / SIM_FIX),
                         (float)((double)(long long)rec[2 * i + 1] / SIM_FIX));
}

}  // namespace

hipError_t launch_simulate(af_ctx* c, int n_scat, const double* scat_xz, const float* amp, int nx,
                           int nz, double x0, double z0, double dx, double dz, const float* s_true,
                           int n_seg, double fc, double frac_bw, float2* iq) {
  // host-side geometry of the scatterers: polar (rho, sin, cos) for the arc lens,
  // (x, z) for the flat one
  std::vector<double4> spol(n_scat);
  std::vector<float2> sxy(n_scat);
  for (int k = 0; k < n_scat; ++k) {
    const double x = scat_xz[2 * k], z = scat_xz[2 * k + 1];
    const double rho = std::sqrt(x * x + z * z);
    spol[k] = c->flat ? make_double4(x, z, 0.0, 0.0) : make_double4(rho, x / rho, z / rho, 0.0);
    sxy[k] = make_float2((float)x, (float)z);
  }
  DBuf d_spol, d_sxy, d_amp, d_T, d_gd, d_sc;
  hipError_t e;
  const size_t gsz = (size_t)(nx + 3) * (nz + 3);
  if ((e = d_spol.ensure(sizeof(double4) * n_scat)) != hipSuccess) return e;
  if ((e = d_sxy.ensure(sizeof(float2) * n_scat)) != hipSuccess) return e;
  if ((e = d_amp.ensure(sizeof(float) * n_scat)) != hipSuccess) return e;
  if ((e = d_T.ensure(sizeof(double) * (size_t)n_scat * c->N)) != hipSuccess) return e;
  if ((e = d_gd.ensure(sizeof(float) * gsz)) != hipSuccess) return e;
  if ((e = d_sc.ensure(sizeof(double) * 8)) != hipSuccess) return e;
  e = hipMemcpyAsync(d_spol.p, spol.data(), sizeof(double4) * n_scat, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_sxy.p, sxy.data(), sizeof(float2) * n_scat, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_amp.p, amp, sizeof(float) * n_scat, hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return e;
  if ((e = launch_prepare_grid(c, s_true, nx, nz, d_gd.as<float>(), d_sc.as<double>(), 0, nullptr,
                               nullptr)) != hipSuccess)
    return e;
  SimGeo sg{nx, nz, nx + 3, n_seg, (float)x0, (float)z0, (float)(1.0 / dx), (float)(1.0 / dz)};
  // the physical lens with bent rays, whatever lens model the beamformer uses
  Geo g = c->geo();
  g.dlens = c->d_lens_phys;
  g.t_ttp = c->t_ttp_phys;
  hipLaunchKernelGGL(k_sim_times, dim3((n_scat + 255) / 256, c->N), dim3(256), 0, c->stream, g, sg,
                     c->d_elem.as<double4>(), d_spol.as<double4>(), d_sxy.as<float2>(), n_scat,
                     d_gd.as<float>(), d_sc.as<double>(), d_T.as<double>());
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const double sigma = std::sqrt(2.0 * std::log(2.0)) / (M_PI * frac_bw * fc);
  hipLaunchKernelGGL(k_sim_synth, dim3(c->N * c->N), dim3(256), sizeof(unsigned long long) * 2 * c->Ns,
                     c->stream, g, d_T.as<double>(), n_scat, d_amp.as<float>(), sigma, iq);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // temporaries are freed after the stream drains
  e = hipStreamSynchronize(c->stream);
  return e;
}

}  // namespace af
