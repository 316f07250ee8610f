// Learned warm start: 3x3 convolutions (padding 1, stride 1 or 2, NHWC) as
// implicit GEMMs on the gfx950 BF16 matrix cores (v_mfma_f32_32x32x16_bf16,
// FP32 accumulate), forward, backward-data and backward-weight, plus the small
// kernels of the training loop (weight packing, MSE gradient, Adam, feature
// packing, resampling of the polar output onto the slowness grid).
//
// Operand layout of the 32x32x16 MFMA (lane l, element i of the 8-wide inputs,
// element j of the 16-wide accumulator):
//   A[m = l % 32][k = 8 (l / 32) + i],  B[k = 8 (l / 32) + i][n = l % 32],
//   C[m = 8 (j / 4) + 4 (l / 32) + j % 4][n = l % 32].
#include <cstdint>

#include "af_internal.h"

namespace af {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint16_t u16;

struct ConvShape {
  int B, H, W, Cin, Cout, stride, Ho, Wo;
  int Kp;    // 9 Cin rounded up to 16 (forward / weight-gradient K)
  int Ktp;   // 9 Cout rounded up to 16 (backward-data K)
};

__device__ inline __bf16 as_bf16(u16 x) { return __builtin_bit_cast(__bf16, x); }
__device__ inline u16 as_u16(__bf16 x) { return __builtin_bit_cast(u16, x); }
__device__ inline u16 f2bf(float f) { return as_u16((__bf16)f); }

__device__ inline bf16x8 zero8() {
  bf16x8 z;
#pragma unroll
  for (int i = 0; i < 8; ++i) z[i] = as_bf16(0);
  return z;
}

// --- forward ----------------------------------------------------------------------
// A[m = output pixel][k = tap * Cin + ci] = in[pixel shifted by tap][ci]
__device__ inline bf16x8 fwd_a(const ConvShape& s, const u16* __restrict__ in, long long p, int k0) {
  const long long M = (long long)s.B * s.Ho * s.Wo;
  if (p >= M) return zero8();
  const int xo = (int)(p % s.Wo);
  const long long t = p / s.Wo;
  const int yo = (int)(t % s.Ho);
  const int b = (int)(t / s.Ho);
  if ((s.Cin & 7) == 0) {
    const int tap = k0 / s.Cin, ci0 = k0 - tap * s.Cin;
    if (tap >= 9) return zero8();
    const int yi = yo * s.stride + tap / 3 - 1, xi = xo * s.stride + tap % 3 - 1;
    if (yi < 0 || yi >= s.H || xi < 0 || xi >= s.W) return zero8();
    return *reinterpret_cast<const bf16x8*>(in + (((long long)b * s.H + yi) * s.W + xi) * s.Cin + ci0);
  }
  bf16x8 v = zero8();
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = k0 + i;
    const int tap = k / s.Cin, ci = k - tap * s.Cin;
    if (tap >= 9) continue;
    const int yi = yo * s.stride + tap / 3 - 1, xi = xo * s.stride + tap % 3 - 1;
    if (yi < 0 || yi >= s.H || xi < 0 || xi >= s.W) continue;
    v[i] = as_bf16(in[(((long long)b * s.H + yi) * s.W + xi) * s.Cin + ci]);
  }
  return v;
}

__global__ __launch_bounds__(256) void k_conv_fwd(ConvShape s, const u16* __restrict__ in,
                                                  const u16* __restrict__ wp,
                                                  const float* __restrict__ bias, int relu,
                                                  u16* __restrict__ out, float* __restrict__ outf) {
  const int l = threadIdx.x & 63;
  const long long base = (long long)blockIdx.x * 128 + (threadIdx.x >> 6) * 32;
  const int hi = l >> 5, lo = l & 31;
  f32x16 acc = {};
  for (int k0 = 0; k0 < s.Kp; k0 += 16) {
    const bf16x8 a = fwd_a(s, in, base + lo, k0 + 8 * hi);
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(wp + (long long)lo * s.Kp + k0 + 8 * hi);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  const long long M = (long long)s.B * s.Ho * s.Wo;
  const int n = lo;
  if (n >= s.Cout) return;
  const float bn = bias[n];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const long long p = base + 8 * (j >> 2) + 4 * hi + (j & 3);
    if (p >= M) continue;
    float v = acc[j] + bn;
    if (outf) outf[p * s.Cout + n] = v;
    if (relu) v = fmaxf(v, 0.f);
    if (out) out[p * s.Cout + n] = f2bf(v);
  }
}

// --- backward data --------------------------------------------------------------------
// dIn[b][yi][xi][ci] = sum_{tap, co} W[co][tap][ci] dOut[b][yo][xo][co] with
// yi = yo * stride + ky - 1.  A[m = input pixel][k = tap * Cout + co].
__device__ inline bf16x8 bwd_a(const ConvShape& s, const u16* __restrict__ dout, long long p, int k0) {
  const long long M = (long long)s.B * s.H * s.W;
  if (p >= M) return zero8();
  const int xi = (int)(p % s.W);
  const long long t = p / s.W;
  const int yi = (int)(t % s.H);
  const int b = (int)(t / s.H);
  bf16x8 v = zero8();
  if ((s.Cout & 7) == 0) {
    const int tap = k0 / s.Cout, co0 = k0 - tap * s.Cout;
    if (tap >= 9) return v;
    const int ny = yi + 1 - tap / 3, nx = xi + 1 - tap % 3;
    if (ny < 0 || nx < 0 || ny % s.stride || nx % s.stride) return v;
    const int yo = ny / s.stride, xo = nx / s.stride;
    if (yo >= s.Ho || xo >= s.Wo) return v;
    return *reinterpret_cast<const bf16x8*>(dout + (((long long)b * s.Ho + yo) * s.Wo + xo) * s.Cout + co0);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = k0 + i;
    const int tap = k / s.Cout, co = k - tap * s.Cout;
    if (tap >= 9) continue;
    const int ny = yi + 1 - tap / 3, nx = xi + 1 - tap % 3;
    if (ny < 0 || nx < 0 || ny % s.stride || nx % s.stride) continue;
    const int yo = ny / s.stride, xo = nx / s.stride;
    if (yo >= s.Ho || xo >= s.Wo) continue;
    v[i] = as_bf16(dout[(((long long)b * s.Ho + yo) * s.Wo + xo) * s.Cout + co]);
  }
  return v;
}

__global__ __launch_bounds__(256) void k_conv_bwd_data(ConvShape s, const u16* __restrict__ dout,
                                                       const u16* __restrict__ wtp,
                                                       const u16* __restrict__ act,
                                                       u16* __restrict__ din) {
  const int l = threadIdx.x & 63;
  const long long base = (long long)blockIdx.x * 128 + (threadIdx.x >> 6) * 32;
  const int hi = l >> 5, lo = l & 31;
  f32x16 acc = {};
  for (int k0 = 0; k0 < s.Ktp; k0 += 16) {
    const bf16x8 a = bwd_a(s, dout, base + lo, k0 + 8 * hi);
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(wtp + (long long)lo * s.Ktp + k0 + 8 * hi);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  const long long M = (long long)s.B * s.H * s.W;
  const int n = lo;
  if (n >= s.Cin) return;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const long long p = base + 8 * (j >> 2) + 4 * hi + (j & 3);
    if (p >= M) continue;
    float v = acc[j];
    // ReLU of the layer below: its output was positive where the gradient passes
    if (act && !((float)as_bf16(act[p * s.Cin + n]) > 0.f)) v = 0.f;
    din[p * s.Cin + n] = f2bf(v);
  }
}

// --- backward weight ------------------------------------------------------------------
// dW[co][kw] = sum_pixels dOut[p][co] in[p shifted by tap(kw)][ci(kw)]:
// GEMM with M = Cout (32), N = Kp (tiles of 32), K = the workgroup's pixels.
__global__ __launch_bounds__(256) void k_conv_bwd_weight(ConvShape s, const u16* __restrict__ in,
                                                         const u16* __restrict__ dout,
                                                         int pix_per_wg, float* __restrict__ part,
                                                         float* __restrict__ bpart) {
  const int l = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int hi = l >> 5, lo = l & 31;
  const long long M = (long long)s.B * s.Ho * s.Wo;
  const long long p_beg = (long long)blockIdx.x * pix_per_wg;
  const long long p_end = min(M, p_beg + pix_per_wg);
  const int n_tiles = s.Kp / 32 + ((s.Kp % 32) ? 1 : 0);
  float* mypart = part + (long long)blockIdx.x * 32 * (n_tiles * 32);
  for (int tile = wave; tile < n_tiles; tile += 4) {
    f32x16 acc = {};
    const int kw = tile * 32 + lo;            // weight column of this lane (B operand)
    const int tap = kw / s.Cin, ci = kw - tap * s.Cin;
    const bool kw_ok = tap < 9 && kw < s.Kp;
    for (long long p0 = p_beg; p0 < p_end; p0 += 16) {
      bf16x8 a = zero8(), b = zero8();
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const long long p = p0 + 8 * hi + i;
        if (p >= p_end) continue;
        if (lo < s.Cout) a[i] = as_bf16(dout[p * s.Cout + lo]);
        if (kw_ok) {
          const int xo = (int)(p % s.Wo);
          const long long t = p / s.Wo;
          const int yo = (int)(t % s.Ho);
          const int bb = (int)(t / s.Ho);
          const int yi = yo * s.stride + tap / 3 - 1, xi = xo * s.stride + tap % 3 - 1;
          if (yi >= 0 && yi < s.H && xi >= 0 && xi < s.W)
            b[i] = as_bf16(in[(((long long)bb * s.H + yi) * s.W + xi) * s.Cin + ci]);
        }
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int m = 8 * (j >> 2) + 4 * hi + (j & 3);   // output channel
      mypart[(long long)m * (n_tiles * 32) + tile * 32 + lo] = acc[j];
    }
  }
  // bias gradient partials: sum of dOut over this workgroup's pixels
  if (threadIdx.x < 32) {
    float sb = 0.f;
    if ((int)threadIdx.x < s.Cout)
      for (long long p = p_beg; p < p_end; ++p) sb += (float)as_bf16(dout[p * s.Cout + threadIdx.x]);
    bpart[(long long)blockIdx.x * 32 + threadIdx.x] = sb;
  }
}

// dW[co][k] (k < 9 Cin) and dbias: fixed-order sums of the workgroup partials.
__global__ __launch_bounds__(256) void k_conv_wreduce(const float* __restrict__ part,
                                                      const float* __restrict__ bpart, int n_wg,
                                                      int cols, int cout, int kvalid,
                                                      float* __restrict__ dw,
                                                      float* __restrict__ db) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx < cout * kvalid) {
    const int co = idx / kvalid, k = idx - co * kvalid;
    float s = 0.f;
    for (int w = 0; w < n_wg; ++w) s += part[((long long)w * 32 + co) * cols + k];
    dw[idx] = s;
  }
  if (idx < cout) {
    float s = 0.f;
    for (int w = 0; w < n_wg; ++w) s += bpart[(long long)w * 32 + idx];
    db[idx] = s;
  }
}

// Pack FP32 weights [Cout][9 Cin] into the BF16 B operands of the forward
// ([32][Kp], row = co) and of the backward-data pass ([32][Ktp], row = ci,
// column = tap * Cout + co); padding is zero.
__global__ __launch_bounds__(256) void k_conv_pack(int Cin, int Cout, int Kp, int Ktp,
                                                   const float* __restrict__ w,
                                                   u16* __restrict__ wp, u16* __restrict__ wtp) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx < 32 * Kp) {
    const int co = idx / Kp, k = idx - co * Kp;
    const float v = (co < Cout && k < 9 * Cin) ? w[co * 9 * Cin + k] : 0.f;
    wp[idx] = f2bf(v);
  }
  if (wtp && idx < 32 * Ktp) {
    const int ci = idx / Ktp, k = idx - ci * Ktp;
    float v = 0.f;
    if (ci < Cin && k < 9 * Cout) {
      const int tap = k / Cout, co = k - tap * Cout;
      v = w[co * 9 * Cin + tap * Cin + ci];
    }
    wtp[idx] = f2bf(v);
  }
}

// loss += sum (out - label)^2 * scale; dOut = 2 (out - label) scale (BF16).
__global__ __launch_bounds__(256) void k_mse(int n, const float* __restrict__ out,
                                             const float* __restrict__ label, float scale,
                                             float* __restrict__ loss, u16* __restrict__ dout) {
  __shared__ float red[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  float e = 0.f;
  if (i < n) {
    const float d = out[i] - label[i];
    e = d * d * scale;
    dout[i] = f2bf(2.f * d * scale);
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_adam_vec(int n, float lr, float b1, float b2, float eps,
                                                  float bc1, float bc2, float* __restrict__ p,
                                                  float* __restrict__ m, float* __restrict__ v,
                                                  const float* __restrict__ g) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Feature maps [C][n] (FP32, channel-major) -> NHWC BF16 [n][C] with per-channel
// affine normalisation (x - shift[c]) * scale[c].
__global__ __launch_bounds__(256) void k_features(long long n, int C, const float* __restrict__ maps,
                                                  const float* __restrict__ shift,
                                                  const float* __restrict__ scale,
                                                  u16* __restrict__ out) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < C; ++c) out[i * C + c] = f2bf((maps[c * n + i] - shift[c]) * scale[c]);
}

// Slowness grid from a polar map: s[i][j] = s_base + scale * bilinear(map) at the
// node's (radius, angle), clamped to the map; map rows are radii r0 + a dr,
// columns angles t0 + b dt.
__global__ __launch_bounds__(256) void k_polar_to_grid(const float* __restrict__ map, int nr, int nt,
                                                       double r0, double dr, double t0, double dt,
                                                       int nx, int nz, double x0, double z0,
                                                       double dx, double dz, float s_base,
                                                       float scale, float* __restrict__ s) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nx * nz) return;
  const int i = idx / nx, j = idx - i * nx;
  const double x = x0 + j * dx, z = z0 + i * dz;
  const double rr = (sqrt(x * x + z * z) - r0) / dr;
  const double tt = (atan2(x, z) - t0) / dt;
  const float u = fminf(fmaxf((float)rr, 0.f), (float)(nr - 1));
  const float v = fminf(fmaxf((float)tt, 0.f), (float)(nt - 1));
  const int a0 = min((int)u, nr - 2), b0 = min((int)v, nt - 2);
  const float fu = u - a0, fv = v - b0;
  const float m00 = map[a0 * nt + b0], m01 = map[a0 * nt + b0 + 1];
  const float m10 = map[(a0 + 1) * nt + b0], m11 = map[(a0 + 1) * nt + b0 + 1];
  const float val = (1 - fu) * ((1 - fv) * m00 + fv * m01) + fu * ((1 - fv) * m10 + fv * m11);
  s[idx] = s_base + scale * val;
}

ConvShape shape(int B, int H, int W, int Cin, int Cout, int stride) {
  ConvShape s;
  s.B = B;
  s.H = H;
  s.W = W;
  s.Cin = Cin;
  s.Cout = Cout;
  s.stride = stride;
  s.Ho = (H - 1) / stride + 1;
  s.Wo = (W - 1) / stride + 1;
  s.Kp = (9 * Cin + 15) / 16 * 16;
  s.Ktp = (9 * Cout + 15) / 16 * 16;
  return s;
}

}  // namespace

hipError_t launch_conv_fwd(af_ctx* c, int B, int H, int W, int Cin, int Cout, int stride, int relu,
                           const void* in, const void* wp, const float* bias, void* out,
                           float* outf) {
  const ConvShape s = shape(B, H, W, Cin, Cout, stride);
  const long long M = (long long)B * s.Ho * s.Wo;
  hipLaunchKernelGGL(k_conv_fwd, dim3((unsigned)((M + 127) / 128)), dim3(256), 0, c->stream, s,
                     (const u16*)in, (const u16*)wp, bias, relu, (u16*)out, outf);
  return hipGetLastError();
}

hipError_t launch_conv_bwd_data(af_ctx* c, int B, int H, int W, int Cin, int Cout, int stride,
                                const void* dout, const void* wtp, const void* act, void* din) {
  const ConvShape s = shape(B, H, W, Cin, Cout, stride);
  const long long M = (long long)B * H * W;
  hipLaunchKernelGGL(k_conv_bwd_data, dim3((unsigned)((M + 127) / 128)), dim3(256), 0, c->stream, s,
                     (const u16*)dout, (const u16*)wtp, (const u16*)act, (u16*)din);
  return hipGetLastError();
}

hipError_t launch_conv_bwd_weight(af_ctx* c, int B, int H, int W, int Cin, int Cout, int stride,
                                  const void* in, const void* dout, float* dw, float* db) {
  const ConvShape s = shape(B, H, W, Cin, Cout, stride);
  const long long M = (long long)B * s.Ho * s.Wo;
  const int pix_per_wg = 2048;
  const int n_wg = (int)((M + pix_per_wg - 1) / pix_per_wg);
  const int n_tiles = s.Kp / 32 + ((s.Kp % 32) ? 1 : 0);
  const int cols = n_tiles * 32;
  hipError_t e = c->d_cnn_part.ensure(sizeof(float) * ((size_t)n_wg * 32 * cols + (size_t)n_wg * 32));
  if (e != hipSuccess) return e;
  float* part = c->d_cnn_part.as<float>();
  float* bpart = part + (size_t)n_wg * 32 * cols;
  hipLaunchKernelGGL(k_conv_bwd_weight, dim3(n_wg), dim3(256), 0, c->stream, s, (const u16*)in,
                     (const u16*)dout, pix_per_wg, part, bpart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int n = Cout * 9 * Cin;
  hipLaunchKernelGGL(k_conv_wreduce, dim3((n + 255) / 256), dim3(256), 0, c->stream, part, bpart,
                     n_wg, cols, Cout, 9 * Cin, dw, db);
  return hipGetLastError();
}

hipError_t launch_conv_pack(af_ctx* c, int Cin, int Cout, const float* w, void* wp, void* wtp) {
  const int Kp = (9 * Cin + 15) / 16 * 16, Ktp = (9 * Cout + 15) / 16 * 16;
  const int n = 32 * (Kp > Ktp ? Kp : Ktp);
  hipLaunchKernelGGL(k_conv_pack, dim3((n + 255) / 256), dim3(256), 0, c->stream, Cin, Cout, Kp, Ktp,
                     w, (u16*)wp, (u16*)wtp);
  return hipGetLastError();
}

hipError_t launch_mse(af_ctx* c, int n, const float* out, const float* label, float scale,
                      float* loss_parts, void* dout) {
  hipLaunchKernelGGL(k_mse, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, out, label, scale,
                     loss_parts, (u16*)dout);
  return hipGetLastError();
}

hipError_t launch_adam_vec(af_ctx* c, int n, const af_adam_params* ap, int step, float* p, float* m,
                           float* v, const float* g) {
  const float bc1 = 1.f - powf(ap->beta1, (float)step), bc2 = 1.f - powf(ap->beta2, (float)step);
  hipLaunchKernelGGL(k_adam_vec, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, ap->lr, ap->beta1,
                     ap->beta2, ap->eps, bc1, bc2, p, m, v, g);
  return hipGetLastError();
}

hipError_t launch_features(af_ctx* c, long long n, int C, const float* maps, const float* shift,
                           const float* scale, void* out) {
  hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, C,
                     maps, shift, scale, (u16*)out);
  return hipGetLastError();
}

hipError_t launch_polar_to_grid(af_ctx* c, const float* map, int nr, int nt, double r0, double dr,
                                double t0, double dt, int nx, int nz, double x0, double z0,
                                double dx, double dz, float s_base, float scale, float* s) {
  hipLaunchKernelGGL(k_polar_to_grid, dim3((nx * nz + 255) / 256), dim3(256), 0, c->stream, map, nr,
                     nt, r0, dr, t0, dt, nx, nz, x0, z0, dx, dz, s_base, scale, s);
  return hipGetLastError();
}

}  // namespace af
