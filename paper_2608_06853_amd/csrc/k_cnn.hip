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
#include <algorithm>
#include <climits>
#include <cstdint>
#include <mutex>

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

// Pixel p = (b * rows + y) * cols + x of a B x rows x cols image, split once per
// lane; valid = false past the last pixel.
struct Pix {
  bool valid;
  int b, y, x;
};
__device__ inline Pix split_pixel(long long p, int B, int rows, int cols) {
  Pix q{false, 0, 0, 0};
  if (p >= (long long)B * rows * cols) return q;
  const long long t = p / cols;
  q.valid = true;
  q.x = (int)(p - t * cols);
  q.b = (int)(t / rows);
  q.y = (int)(t - (long long)q.b * rows);
  return q;
}

// acc += sum over K-steps k = 0, 16, .., K - 16 of W[:, k..k+15] X[k..k+15, :] (the
// weight row of this lane at wrow, the pixel operand from opnd(k)).  The loads of U
// K-steps are issued before their MFMAs so that U are in flight per wave; steps past
// the end load the last step again and skip its MFMA.
template <int U, class Op>
__device__ inline f32x16 kloop(int K, const u16* __restrict__ wrow, f32x16 acc, Op opnd) {
  for (int k0 = 0; k0 < K; k0 += 16 * U) {
    bf16x8 w[U], x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = min(k0 + 16 * u, K - 16);
      w[u] = *reinterpret_cast<const bf16x8*>(wrow + k);
      x[u] = opnd(k);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k0 + 16 * u < K) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[u], x[u], acc, 0, 0, 0);
  }
  return acc;
}

// Buffer resource over a tensor of `bytes` (below 2 GiB): a raw buffer load at a
// byte offset at or past the end returns zero instead of faulting, which makes the
// padding taps free of branches.  Word 3 = 0x00020000 (32-bit data format), the value
// for raw buffer access on gfx9-family chips.
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr uint32_t OOB = 0x80000000u;    // past every record (tensors are below 2 GiB)
__device__ inline Rsrc make_rsrc(const void* p, long long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// --- forward ----------------------------------------------------------------------
// Im2col operand X[pixel][k = tap * Cin + ci] = in[pixel shifted by tap][ci]: the 8
// values k0 .. k0 + 7 of output pixel q.
// Branch-free: a lane whose tap falls outside the image loads element 0 and keeps
// zero, so the loads of several K-steps can be in flight together.
// fwd_v: Cin a multiple of 8, one 16-byte load; fwd_e: element by element.
__device__ inline bf16x8 fwd_v(const ConvShape& s, Rsrc in, const Pix& q, int k0) {
  const int tap = k0 / s.Cin, ci0 = k0 - tap * s.Cin;
  const int yi = q.y * s.stride + tap / 3 - 1, xi = q.x * s.stride + tap % 3 - 1;
  const bool ok = q.valid & (tap < 9) & (yi >= 0) & (yi < s.H) & (xi >= 0) & (xi < s.W);
  const uint32_t e = (((uint32_t)q.b * s.H + (uint32_t)yi) * s.W + (uint32_t)xi) * s.Cin + ci0;
  return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(in, ok ? 2 * e : OOB, 0, 0));
}
__device__ inline bf16x8 fwd_e(const ConvShape& s, Rsrc in, const Pix& q, int k0) {
  bf16x8 v;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = k0 + i;
    const int tap = k / s.Cin, ci = k - tap * s.Cin;
    const int yi = q.y * s.stride + tap / 3 - 1, xi = q.x * s.stride + tap % 3 - 1;
    const bool ok = q.valid & (tap < 9) & (yi >= 0) & (yi < s.H) & (xi >= 0) & (xi < s.W);
    const uint32_t e = (((uint32_t)q.b * s.H + (uint32_t)yi) * s.W + (uint32_t)xi) * s.Cin + ci;
    v[i] = as_bf16(__builtin_amdgcn_raw_buffer_load_b16(in, ok ? 2 * e : OOB, 0, 0));
  }
  return v;
}

// fwd_c2: Cin = 2 (the first layer): the values k0 .. k0 + 7 are taps k0 / 2 .. k0 / 2 + 3
// with both channels each, so four 4-byte loads.
__device__ inline bf16x8 fwd_c2(const ConvShape& s, Rsrc in, const Pix& q, int k0) {
  bf16x8 v;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int tap = (k0 >> 1) + j;
    const int yi = q.y * s.stride + tap / 3 - 1, xi = q.x * s.stride + tap % 3 - 1;
    const bool ok = q.valid & (tap < 9) & (yi >= 0) & (yi < s.H) & (xi >= 0) & (xi < s.W);
    const uint32_t e = (((uint32_t)q.b * s.H + (uint32_t)yi) * s.W + (uint32_t)xi) * 2u;
    const uint32_t d = __builtin_amdgcn_raw_buffer_load_b32(in, ok ? 2 * e : OOB, 0, 0);
    v[2 * j] = as_bf16((u16)(d & 0xffffu));
    v[2 * j + 1] = as_bf16((u16)(d >> 16));
  }
  return v;
}

// The product is taken transposed, C[m = co][n = pixel] = W X^T, so that a lane's
// accumulators are channels 8q + 4 (l / 32) + 0..3 (q = 0..3) of one pixel: each
// group of four is one 8-byte store.
__global__ __launch_bounds__(256) void k_conv_fwd(ConvShape s, const u16* __restrict__ in,
                                                  const u16* __restrict__ wp,
                                                  const float* __restrict__ bias, int relu,
                                                  u16* __restrict__ out, float* __restrict__ outf) {
  const int l = threadIdx.x & 63;
  const long long base = (long long)blockIdx.x * 128 + (threadIdx.x >> 6) * 32;
  const int hi = l >> 5, lo = l & 31;
  const Pix q = split_pixel(base + lo, s.B, s.Ho, s.Wo);
  const Rsrc rin = make_rsrc(in, 2LL * s.B * s.H * s.W * s.Cin);
  const u16* wrow = wp + (long long)lo * s.Kp + 8 * hi;
  f32x16 acc = {};
  if ((s.Cin & 7) == 0)
    acc = kloop<6>(s.Kp, wrow, acc, [&](int k) { return fwd_v(s, rin, q, k + 8 * hi); });
  else if (s.Cin == 2)
    acc = kloop<2>(s.Kp, wrow, acc, [&](int k) { return fwd_c2(s, rin, q, k + 8 * hi); });
  else
    acc = kloop<2>(s.Kp, wrow, acc, [&](int k) { return fwd_e(s, rin, q, k + 8 * hi); });
  const long long M = (long long)s.B * s.Ho * s.Wo;
  const long long p = base + lo;
  if (p >= M) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c0 = 8 * q + 4 * hi;
    if (c0 >= s.Cout) continue;
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = acc[4 * q + r] + (c0 + r < s.Cout ? bias[c0 + r] : 0.f);
    if (outf) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (c0 + r < s.Cout) outf[p * s.Cout + c0 + r] = v[r];
    }
    if (!out) continue;
    if (relu) {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = fmaxf(v[r], 0.f);
    }
    if ((s.Cout & 3) == 0) {
      uint2 w2;
      w2.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
      w2.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
      *reinterpret_cast<uint2*>(out + p * s.Cout + c0) = w2;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (c0 + r < s.Cout) out[p * s.Cout + c0 + r] = f2bf(v[r]);
    }
  }
}

// --- backward data --------------------------------------------------------------------
// dIn[b][yi][xi][ci] = sum_{tap, co} W[co][tap][ci] dOut[b][yo][xo][co] with
// yi = yo * stride + ky - 1.  Operand dOut[input pixel][k = tap * Cout + co].
// bwd_v: Cout a multiple of 8, one 16-byte load; bwd_e: element by element.  The
// stride is 1 or 2, so the parity test and the halving are bit operations.
__device__ inline bf16x8 bwd_v(const ConvShape& s, Rsrc dout, const Pix& q, int k0) {
  const int tap = k0 / s.Cout, co0 = k0 - tap * s.Cout;
  const int ny = q.y + 1 - tap / 3, nx = q.x + 1 - tap % 3;
  const int sh = s.stride - 1;
  const int yo = ny >> sh, xo = nx >> sh;
  const bool ok = q.valid & (tap < 9) & (ny >= 0) & (nx >= 0) & (((ny | nx) & sh) == 0) &
                  (yo < s.Ho) & (xo < s.Wo);
  const uint32_t e = (((uint32_t)q.b * s.Ho + (uint32_t)yo) * s.Wo + (uint32_t)xo) * s.Cout + co0;
  return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(dout, ok ? 2 * e : OOB, 0, 0));
}
__device__ inline bf16x8 bwd_e(const ConvShape& s, Rsrc dout, const Pix& q, int k0) {
  bf16x8 v;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = k0 + i;
    const int tap = k / s.Cout, co = k - tap * s.Cout;
    const int ny = q.y + 1 - tap / 3, nx = q.x + 1 - tap % 3;
    const int sh = s.stride - 1;
    const int yo = ny >> sh, xo = nx >> sh;
    const bool ok = q.valid & (tap < 9) & (ny >= 0) & (nx >= 0) & (((ny | nx) & sh) == 0) &
                    (yo < s.Ho) & (xo < s.Wo);
    const uint32_t e = (((uint32_t)q.b * s.Ho + (uint32_t)yo) * s.Wo + (uint32_t)xo) * s.Cout + co;
    v[i] = as_bf16(__builtin_amdgcn_raw_buffer_load_b16(dout, ok ? 2 * e : OOB, 0, 0));
  }
  return v;
}

// Transposed like the forward: C[m = ci][n = input pixel], four channels per store.
__global__ __launch_bounds__(256) void k_conv_bwd_data(ConvShape s, const u16* __restrict__ dout,
                                                       const u16* __restrict__ wtp,
                                                       const u16* __restrict__ act,
                                                       u16* __restrict__ din) {
  const int l = threadIdx.x & 63;
  const long long base = (long long)blockIdx.x * 128 + (threadIdx.x >> 6) * 32;
  const int hi = l >> 5, lo = l & 31;
  const Pix q = split_pixel(base + lo, s.B, s.H, s.W);
  const Rsrc rdo = make_rsrc(dout, 2LL * s.B * s.Ho * s.Wo * s.Cout);
  const u16* wrow = wtp + (long long)lo * s.Ktp + 8 * hi;
  f32x16 acc = {};
  if ((s.Cout & 7) == 0)
    acc = kloop<6>(s.Ktp, wrow, acc, [&](int k) { return bwd_v(s, rdo, q, k + 8 * hi); });
  else
    acc = kloop<2>(s.Ktp, wrow, acc, [&](int k) { return bwd_e(s, rdo, q, k + 8 * hi); });
  const long long M = (long long)s.B * s.H * s.W;
  const long long p = base + lo;
  if (p >= M) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c0 = 8 * q + 4 * hi;
    if (c0 >= s.Cin) continue;
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = acc[4 * q + r];
    const long long o = p * s.Cin + c0;
    // ReLU of the layer below: its output was positive where the gradient passes
    if ((s.Cin & 3) == 0) {
      if (act) {
        const uint2 a2 = *reinterpret_cast<const uint2*>(act + o);
        const uint32_t aw[2] = {a2.x, a2.y};
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (!((float)as_bf16((u16)(aw[r >> 1] >> (16 * (r & 1)))) > 0.f)) v[r] = 0.f;
      }
      uint2 w2;
      w2.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
      w2.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
      *reinterpret_cast<uint2*>(din + o) = w2;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (c0 + r >= s.Cin) continue;
        if (act && !((float)as_bf16(act[o + r]) > 0.f)) v[r] = 0.f;
        din[o + r] = f2bf(v[r]);
      }
    }
  }
}

// Stride 2 with Cout a multiple of 16: wave w of a workgroup takes the input pixels
// of parity class (y mod 2, x mod 2) = (w / 2, w % 2) at 32 consecutive positions
// (b, i, j) of the half-resolution grid, pixel (2 i + y mod 2, 2 j + x mod 2), so the
// four waves cover the same 2 x 64 patch and complete its cache lines together.
// Only taps with y + 1 - ky and x + 1 - kx even reach an output pixel, so the class
// fixes them for the whole wave: ky = 1 for even rows, ky in {0, 2} for odd rows
// (likewise kx), 1, 2 or 4 taps instead of 9.  Each tap spans Cout / 16 whole
// K-steps of the packed weights.
__global__ __launch_bounds__(256) void k_conv_bwd_data_s2(ConvShape s,
                                                          const u16* __restrict__ dout,
                                                          const u16* __restrict__ wtp,
                                                          const u16* __restrict__ act,
                                                          u16* __restrict__ din) {
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int hi = l >> 5, lo = l & 31;
  const int py = wave >> 1, px = wave & 1;
  const int Hc = (s.H + 1) >> 1, Wc = (s.W + 1) >> 1;
  const Pix qc = split_pixel((long long)blockIdx.x * 32 + lo, s.B, Hc, Wc);
  const int y = py + 2 * qc.y, x = px + 2 * qc.x;
  const bool valid = qc.valid & (y < s.H) & (x < s.W);
  const Rsrc rdo = make_rsrc(dout, 2LL * s.B * s.Ho * s.Wo * s.Cout);
  const u16* wrow = wtp + (long long)lo * s.Ktp + 8 * hi;
  const int nsub = s.Cout >> 4;           // K-steps per tap (1 or 2)
  bf16x8 w[8], d[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {           // i = (tap a, tap b, K-step of the tap)
    const int a = i >> 2, b = (i >> 1) & 1, sub = i & 1;
    const bool use = (a <= py) & (b <= px) & (sub < nsub);
    const int ky = py ? 2 * a : 1, kx = px ? 2 * b : 1;
    const int k0 = (3 * ky + kx) * s.Cout + 16 * sub;
    const int yo = (y + 1 - ky) >> 1, xo = (x + 1 - kx) >> 1;   // y + 1 - ky >= 0 in every class
    const bool ok = use & valid & (yo < s.Ho) & (xo < s.Wo);
    const uint32_t e = (((uint32_t)qc.b * s.Ho + (uint32_t)yo) * s.Wo + (uint32_t)xo) * s.Cout +
                       16 * sub + 8 * hi;
    w[i] = *reinterpret_cast<const bf16x8*>(wrow + (use ? k0 : 0));
    d[i] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rdo, ok ? 2 * e : OOB, 0, 0));
  }
  f32x16 acc = {};
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int a = i >> 2, b = (i >> 1) & 1, sub = i & 1;
    if ((a <= py) & (b <= px) & (sub < nsub))
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[i], d[i], acc, 0, 0, 0);
  }
  if (!valid) return;
  const long long p = ((long long)qc.b * s.H + y) * s.W + x;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c0 = 8 * q + 4 * hi;
    if (c0 >= s.Cin) continue;
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = acc[4 * q + r];
    const long long o = p * s.Cin + c0;
    if ((s.Cin & 3) == 0) {
      if (act) {
        const uint2 a2 = *reinterpret_cast<const uint2*>(act + o);
        const uint32_t aw[2] = {a2.x, a2.y};
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (!((float)as_bf16((u16)(aw[r >> 1] >> (16 * (r & 1)))) > 0.f)) v[r] = 0.f;
      }
      uint2 w2;
      w2.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
      w2.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
      *reinterpret_cast<uint2*>(din + o) = w2;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (c0 + r >= s.Cin) continue;
        if (act && !((float)as_bf16(act[o + r]) > 0.f)) v[r] = 0.f;
        din[o + r] = f2bf(v[r]);
      }
    }
  }
}

// --- backward weight ------------------------------------------------------------------
// dW[co][kw] = sum over output pixels p of dOut[p][co] X[p][kw], where X[p][kw] is the
// input under tap(kw) of pixel p: a GEMM with M = Cout (32), N = Kp in tiles of 32 and
// K = pixels.  The matrix cores want 8 consecutive K values per lane, but both
// operands are stored channel-fastest, so a workgroup stages chunks of 64 output
// pixels in LDS transposed (pixel fastest): dOut^T [co][p] and X^T [kw][p].  One
// 16-byte LDS read then gives a lane its 8 pixels of either operand.  Global loads
// are 16 bytes (8 channels of one pixel) when the channel count allows it.
constexpr int WB_CHUNK = 64;             // output pixels per staged chunk (4 MFMA K-steps)
constexpr int WB_LD = WB_CHUNK + 8;      // LDS row stride in BF16 values (16 B of padding)
constexpr int WB_ROWS = 288;             // X^T rows: Kp of the widest layer (Cin = 32)
constexpr int WB_MAX_WG = 768;           // three workgroups per CU fit in LDS
constexpr int WB_GROUPS = 32;            // partial groups of the first reduce pass

__device__ inline bf16x8 lds8(const u16* p) { return *reinterpret_cast<const bf16x8*>(p); }

// Each workgroup accumulates over the chunks blockIdx.x, blockIdx.x + gridDim.x, ...
// With four or more weight tiles each wave owns whole tiles (tiles wave, wave + 4,
// wave + 8) over all K-steps; with fewer, the waves split the K-steps of every tile
// and their sums are added in LDS.  The workgroup writes one partial slab: the
// [32][cols] weight block followed by the 32 bias sums.
__global__ __launch_bounds__(256) void k_conv_bwd_weight(ConvShape s, const u16* __restrict__ in,
                                                         const u16* __restrict__ dout,
                                                         int n_chunks, float* __restrict__ part) {
  __shared__ __align__(16) u16 DT[32 * WB_LD];
  __shared__ __align__(16) u16 XT[WB_ROWS * WB_LD];
  const int tid = threadIdx.x, l = tid & 63, wave = tid >> 6;
  const int hi = l >> 5, lo = l & 31;
  const long long M = (long long)s.B * s.Ho * s.Wo;
  const int n_tiles = (s.Kp + 31) / 32, cols = n_tiles * 32;
  const int kval = 9 * s.Cin;
  const bool split = n_tiles < 4;
  // rows that no chunk writes (channels past Cout, columns past 9 Cin) stay zero
  for (int i = tid; i < (32 - s.Cout) * WB_LD; i += 256) DT[s.Cout * WB_LD + i] = 0;
  for (int i = tid; i < (cols - kval) * WB_LD; i += 256) XT[kval * WB_LD + i] = 0;

  f32x16 acc[3] = {};
  float bsum = 0.f;
  const int pp = l;        // staging: lane = pixel of the chunk, wave = channel group
  for (int ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
    const long long p = (long long)ch * WB_CHUNK + pp;
    const bool pv = p < M;
    int yo = 0, xo = 0;
    long long pix = 0;     // input pixel under the centre tap
    if (pv) {
      xo = (int)(p % s.Wo);
      const long long t = p / s.Wo;
      yo = (int)(t % s.Ho);
      pix = ((t / s.Ho) * s.H + (long long)yo * s.stride) * s.W + (long long)xo * s.stride;
    }
    unsigned okm = 0;      // taps whose input pixel lies inside the image
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int yi = yo * s.stride + tap / 3 - 1, xi = xo * s.stride + tap % 3 - 1;
      if (pv && yi >= 0 && yi < s.H && xi >= 0 && xi < s.W) okm |= 1u << tap;
    }
    __syncthreads();       // the previous chunk's operands have been read
    // all nine taps of a channel group are loaded before any is stored
    if ((s.Cout & 7) == 0) {
      for (int g = wave; g < (s.Cout >> 3); g += 4) {
        const bf16x8 v = pv ? *reinterpret_cast<const bf16x8*>(dout + p * s.Cout + 8 * g) : zero8();
#pragma unroll
        for (int e = 0; e < 8; ++e) DT[(8 * g + e) * WB_LD + pp] = as_u16(v[e]);
      }
    } else {
      for (int c = wave; c < s.Cout; c += 4) DT[c * WB_LD + pp] = pv ? dout[p * s.Cout + c] : (u16)0;
    }
    if ((s.Cin & 7) == 0) {
      for (int g = wave; g < (s.Cin >> 3); g += 4) {
        bf16x8 v[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
          const long long off = (pix + (long long)(tap / 3 - 1) * s.W + (tap % 3 - 1)) * s.Cin;
          v[tap] = (okm >> tap & 1u) ? *reinterpret_cast<const bf16x8*>(in + off + 8 * g) : zero8();
        }
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
#pragma unroll
          for (int e = 0; e < 8; ++e) XT[(tap * s.Cin + 8 * g + e) * WB_LD + pp] = as_u16(v[tap][e]);
      }
    } else {
      for (int ci = wave; ci < s.Cin; ci += 4) {
        u16 v[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
          const long long off = (pix + (long long)(tap / 3 - 1) * s.W + (tap % 3 - 1)) * s.Cin;
          v[tap] = (okm >> tap & 1u) ? in[off + ci] : (u16)0;
        }
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) XT[(tap * s.Cin + ci) * WB_LD + pp] = v[tap];
      }
    }
    __syncthreads();
    if (tid < 32) {        // bias gradient: this chunk's dOut summed per channel
#pragma unroll
      for (int q = 0; q < WB_CHUNK; q += 8) {
        const bf16x8 v = lds8(DT + tid * WB_LD + q);
#pragma unroll
        for (int e = 0; e < 8; ++e) bsum += (float)v[e];
      }
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      if (split && ks != wave) continue;
      const bf16x8 a = lds8(DT + lo * WB_LD + 16 * ks + 8 * hi);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int t = split ? j : wave + 4 * j;
        if (t < n_tiles)
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              a, lds8(XT + (t * 32 + lo) * WB_LD + 16 * ks + 8 * hi), acc[j], 0, 0, 0);
      }
    }
  }
  if (split) {             // waves 1-3 hand their sums to wave 0 through LDS (3 x 3 x 4 KB)
    float* red = reinterpret_cast<float*>(XT);
    __syncthreads();
    if (wave > 0) {
#pragma unroll
      for (int j = 0; j < 3; ++j)
        if (j < n_tiles)
#pragma unroll
          for (int jj = 0; jj < 16; ++jj) red[(((wave - 1) * 3 + j) * 16 + jj) * 64 + l] = acc[j][jj];
    }
    __syncthreads();
    if (wave == 0) {
      for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          if (j < n_tiles)
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) acc[j][jj] += red[((w * 3 + j) * 16 + jj) * 64 + l];
    }
  }
  float* slab = part + (long long)blockIdx.x * (32 * cols + 32);
  if (!split || wave == 0) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int t = split ? j : wave + 4 * j;
      if (t >= n_tiles) continue;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int m = 8 * (jj >> 2) + 4 * hi + (jj & 3);   // output channel
        slab[m * cols + t * 32 + lo] = acc[j][jj];
      }
    }
  }
  if (tid < 32) slab[32 * cols + tid] = bsum;
}

// First reduce pass: slab element e summed over the partials of group blockIdx.y
// (partials per_group * y ... per_group * (y + 1) - 1, in order).
__global__ __launch_bounds__(256) void k_conv_wsum(const float* __restrict__ part, int n_part,
                                                   int per_group, int slab_len,
                                                   float* __restrict__ part2) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= slab_len) return;
  const int w0 = blockIdx.y * per_group, w1 = min(n_part, w0 + per_group);
  float s = 0.f;
#pragma unroll 8
  for (int w = w0; w < w1; ++w) s += part[(long long)w * slab_len + e];  // loads in flight together
  part2[(long long)blockIdx.y * slab_len + e] = s;
}

// Second pass: dW[co][k] (k < 9 Cin) and dbias summed over the groups in order.
__global__ __launch_bounds__(256) void k_conv_wreduce(const float* __restrict__ part2, int n_groups,
                                                      int cols, int cout, int kvalid,
                                                      float* __restrict__ dw,
                                                      float* __restrict__ db) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int slab_len = 32 * cols + 32;
  if (idx < cout * kvalid) {
    const int co = idx / kvalid, k = idx - co * kvalid;
    float s = 0.f;
#pragma unroll 8
    for (int g = 0; g < n_groups; ++g) s += part2[(long long)g * slab_len + co * cols + k];
    dw[idx] = s;
  }
  if (idx < cout) {
    float s = 0.f;
#pragma unroll 8
    for (int g = 0; g < n_groups; ++g) s += part2[(long long)g * slab_len + 32 * cols + idx];
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
// columns angles t0 + b dt; the result is clamped to [s_lo, s_hi].
__global__ __launch_bounds__(256) void k_polar_to_grid(const float* __restrict__ map, int nr, int nt,
                                                       double r0, double dr, double t0, double dt,
                                                       int nx, int nz, double x0, double z0,
                                                       double dx, double dz, float s_base,
                                                       float scale, float s_lo, float s_hi,
                                                       float* __restrict__ s) {
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
  s[idx] = fminf(fmaxf(s_base + scale * val, s_lo), s_hi);  // NaN -> s_lo
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
  if (stride == 2 && (Cout & 15) == 0) {
    const long long mc = (long long)B * ((H + 1) / 2) * ((W + 1) / 2);
    hipLaunchKernelGGL(k_conv_bwd_data_s2, dim3((unsigned)((mc + 31) / 32)), dim3(256), 0,
                       c->stream, s, (const u16*)dout, (const u16*)wtp, (const u16*)act,
                       (u16*)din);
    return hipGetLastError();
  }
  const long long M = (long long)B * H * W;
  hipLaunchKernelGGL(k_conv_bwd_data, dim3((unsigned)((M + 127) / 128)), dim3(256), 0, c->stream, s,
                     (const u16*)dout, (const u16*)wtp, (const u16*)act, (u16*)din);
  return hipGetLastError();
}

namespace {

// Work split of the weight gradient: workgroups, reduce groups and the partial-sum
// floats it needs (one slab per workgroup and per group).
struct WbSplit {
  int n_chunks, n_wg, cols, slab_len, per_group, n_groups;
  size_t floats;
};

bool wb_split(const ConvShape& s, WbSplit& w) {
  const long long M = (long long)s.B * s.Ho * s.Wo;
  const long long n_chunks = (M + WB_CHUNK - 1) / WB_CHUNK;
  if (n_chunks > INT_MAX) return false;
  w.n_chunks = (int)n_chunks;
  // about four chunks per workgroup, at most three workgroups per CU
  w.n_wg = (int)std::min<long long>(WB_MAX_WG, (n_chunks + 3) / 4);
  w.cols = (s.Kp + 31) / 32 * 32;
  w.slab_len = 32 * w.cols + 32;
  w.per_group = (w.n_wg + WB_GROUPS - 1) / WB_GROUPS;
  w.n_groups = (w.n_wg + w.per_group - 1) / w.per_group;
  w.floats = (size_t)(w.n_wg + w.n_groups) * w.slab_len;
  return true;
}

// Partial sums of the no-allocation weight gradient (af_conv3x3_bwd_weight_noalloc):
// the most any layer shape needs -- WB_MAX_WG workgroup slabs and WB_GROUPS group
// slabs, each a 32 x 288 weight block plus 32 bias sums: 800 x 9248 floats, 29.6 MB
// per GPU, held until the process ends.  Every slab element is written before it is
// read, so nothing is cleared between calls.  Host code never uses this name as an
// address: scratch_ptr holds each device's address from hipGetSymbolAddress.
constexpr size_t NOALLOC_FLOATS = (size_t)(WB_MAX_WG + WB_GROUPS) * (32 * WB_ROWS + 32);
__device__ __align__(256) float scratch[NOALLOC_FLOATS];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
float* scratch_ptr[MAX_DEVICES] = {};

hipError_t run_conv_bwd_weight(af_ctx* c, const ConvShape& s, const WbSplit& w, const void* in,
                               const void* dout, float* part, float* dw, float* db) {
  float* part2 = part + (size_t)w.n_wg * w.slab_len;
  hipLaunchKernelGGL(k_conv_bwd_weight, dim3(w.n_wg), dim3(256), 0, c->stream, s, (const u16*)in,
                     (const u16*)dout, w.n_chunks, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_conv_wsum, dim3((w.slab_len + 255) / 256, w.n_groups), dim3(256), 0,
                     c->stream, part, w.n_wg, w.per_group, w.slab_len, part2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int n = s.Cout * 9 * s.Cin;
  hipLaunchKernelGGL(k_conv_wreduce, dim3((n + 255) / 256), dim3(256), 0, c->stream, part2,
                     w.n_groups, w.cols, s.Cout, 9 * s.Cin, dw, db);
  return hipGetLastError();
}

}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;  // this device's copy of the array (the device is current)
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  scratch_ptr[device] = static_cast<float*>(p);
  return hipSuccess;
}

hipError_t launch_conv_bwd_weight_noalloc(af_ctx* c, int B, int H, int W, int Cin, int Cout,
                                          int stride, const void* in, const void* dout, float* dw,
                                          float* db, bool* too_large) {
  *too_large = false;
  const ConvShape s = shape(B, H, W, Cin, Cout, stride);
  WbSplit w;
  if (!wb_split(s, w)) return hipErrorInvalidValue;
  if (w.floats > NOALLOC_FLOATS) {
    *too_large = true;
    return hipErrorInvalidValue;
  }
  float* part = nullptr;
  {
    std::lock_guard<std::mutex> lock(scratch_mu);
    part = (c->device >= 0 && c->device < MAX_DEVICES) ? scratch_ptr[c->device] : nullptr;
  }
  if (!part) return hipErrorNotInitialized;  // af_create could not take the address
  return run_conv_bwd_weight(c, s, w, in, dout, part, dw, db);
}

hipError_t launch_conv_bwd_weight(af_ctx* c, int B, int H, int W, int Cin, int Cout, int stride,
                                  const void* in, const void* dout, float* dw, float* db) {
  const ConvShape s = shape(B, H, W, Cin, Cout, stride);
  WbSplit w;
  if (!wb_split(s, w)) return hipErrorInvalidValue;
  hipError_t e = c->d_cnn_part.ensure(sizeof(float) * w.floats);
  if (e != hipSuccess) return e;
  return run_conv_bwd_weight(c, s, w, in, dout, c->d_cnn_part.as<float>(), dw, db);
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
                                double dx, double dz, float s_base, float scale, float s_lo,
                                float s_hi, float* s) {
  hipLaunchKernelGGL(k_polar_to_grid, dim3((nx * nz + 255) / 256), dim3(256), 0, c->stream, map, nr,
                     nt, r0, dr, t0, dt, nx, nz, x0, z0, dx, dz, s_base, scale, s_lo, s_hi, s);
  return hipGetLastError();
}

}  // namespace af
