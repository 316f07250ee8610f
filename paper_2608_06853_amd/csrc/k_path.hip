// Adjoint of the path integral: dL/ds[node] += sum over rays and ray points of
// dL/dT * L2 * w_k * (bicubic weight of the node at r_k) / N.  Refraction points
// and c_med are held constant (they follow the global mean speed); each ray's
// start and medium leg L2 are read from the table kernel of the same slowness.
//
// A workgroup takes one tile of points and every active element of it; a
// wavefront walks the rays from the elements to its 64 points in lock step.  The
// rays are nearly parallel, so at a given step the lanes usually sit in one grid
// cell.  Every Keys weight is a cubic in its fraction, so the tap sums of ray
// points in one cell are fixed combinations of the 16 moments c g^b f^a (f, g: the
// fractions in the cell, c: the ray point's adjoint weight).  Ray points add their
// moments into registers until the wavefront leaves the cell; then the moments are
// summed across the wavefront with a reduce-scatter, turned into the 16 tap sums
// by the Keys coefficients (lane rotations and row exchanges), and 16 lanes add
// them to an LDS copy of the padded grid with LDS float atomics.  A step whose ray
// points lie in several cells takes one such round per cell.  The rays of four
// neighbouring elements are walked together (pairs or single elements where the
// aperture edge leaves fewer with work).  The copies are summed into one partial
// grid per workgroup, and a second kernel adds the partial grids node by node in a
// fixed order.
#include "af_internal.h"

namespace af {
namespace {

// Cross-lane moves of the reduce-scatter, all on the VALU (no LDS round trip):
// permlane32_swap exchanges the upper half-wave of its first operand with the
// lower half-wave of its second; permlane16_swap does the same for odd rows of
// the first and even rows of the second; the DPP moves read lane l ^ 8
// (row_ror:8), l ^ 7 (row_half_mirror), l ^ 2 and l ^ 1 (quad_perm).
__device__ inline void swap32(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}
__device__ inline void swap16(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}
// (every move used here reads a lane that exists, so bound_ctrl changes no result;
// it lets the compiler fold the move into the instruction that uses it)
template <int CTRL>
__device__ inline float dpp(float x) {
  return __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(x), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ inline int dppi(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xf, 0xf, false);
}
constexpr int DPP_ROR8 = 0x128, DPP_HALF_MIRROR = 0x141, DPP_XOR2 = 0x4e, DPP_XOR1 = 0xb1;
constexpr int DPP_ROR12 = 0x12c, DPP_ROR4 = 0x124;

// Sum over the wavefront of v[i], i = 0..15: every lane returns the sum of
// v[(l >> 2) & 15] (bit 3 of the index is lane bit 5, bit 2 lane bit 4, bit 1
// lane bit 3, bit 0 lane bit 2).  Each stage halves the values a lane holds:
// the half-wave swaps pair lanes l, l ^ 32 and l, l ^ 16 with no selects; the
// last two stages pair l, l ^ 8 and l, l ^ 7 inside rows; a quad all-reduce ends.
__device__ inline float reduce_scatter16(float v[16], int lane) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    swap32(v[i], v[8 + i]);       // lower half: both halves of v[i]; upper: of v[8+i]
    v[i] += v[8 + i];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    swap16(v[i], v[4 + i]);       // rows 0, 2: both rows of v[i]; rows 1, 3: of v[4+i]
    v[i] += v[4 + i];
  }
  const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0;
  float h2[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float send = b3 ? v[i] : v[2 + i];
    const float keep = b3 ? v[2 + i] : v[i];
    h2[i] = keep + dpp<DPP_ROR8>(send);
  }
  const float send = b2 ? h2[0] : h2[1];
  float h1 = (b2 ? h2[1] : h2[0]) + dpp<DPP_HALF_MIRROR>(send);
  h1 += dpp<DPP_XOR2>(h1);
  h1 += dpp<DPP_XOR1>(h1);
  return h1;
}

// Adds v to an LDS grid node with one LDS float atomic (no read-back wait).  On a
// wavefront's private grid copy the lanes of one call hit distinct nodes and the
// calls of a wavefront execute in order, so the sums are deterministic; on a copy
// shared by the workgroup's wavefronts the order of their adds varies.
__device__ inline void lds_add(float* p, float v) { atomicAdd(p, v); }

__device__ inline float readlane_f(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// The value of x in the lane of the same column whose row (lane bits 4-5) differs
// by 1 (exch16) or by 2 (exch32).
__device__ inline float exch16(float x) {
  float a = x, b = x;
  swap16(a, b);  // a: rows 0, 0, 2, 2 of x; b: rows 1, 1, 3, 3
  return (threadIdx.x & 16) ? a : b;
}
__device__ inline float exch32(float x) {
  float a = x, b = x;
  swap32(a, b);  // a: lower half of x twice; b: upper half twice
  return (threadIdx.x & 32) ? a : b;
}

// Coefficient of f^pw in the Keys weight of tap t (nodes j0 - 1 .. j0 + 2) at
// fraction f: the rows of keys_weights written out as polynomials.
__device__ inline float keys_coef(int t, int pw) {
  const float t0 = pw == 1 ? -0.5f : pw == 2 ? 1.0f : pw == 3 ? -0.5f : 0.0f;
  const float t1 = pw == 0 ? 1.0f : pw == 2 ? -2.5f : pw == 3 ? 1.5f : 0.0f;
  const float t2 = pw == 1 ? 0.5f : pw == 2 ? 2.0f : pw == 3 ? -1.5f : 0.0f;
  const float t3 = pw == 2 ? -0.5f : pw == 3 ? 0.5f : 0.0f;
  return t == 0 ? t0 : t == 1 ? t1 : t == 2 ? t2 : t3;
}

// Per-lane coefficients of the moment flush.  After the reduce-scatter lane l holds
// the moment of value index (l >> 2) & 15 = 4 b + a (b: power of the z fraction,
// lane bits 4-5; a: power of the x fraction, lane bits 2-3), and it finishes with
// the tap (r, c) = (b, a) of its own lane position.  kx[d] is the Keys coefficient
// of tap c for the power held by the lane the d-th row rotation reads; kz[d] that of
// tap r for the power held by the lane the d-th row exchange reads.  The sources
// are found by applying the same moves to the lane's own indices.
struct MomentCoef {
  float kx[4], kz0, kz2, kz1s, kz3s;  // kz1s, kz3s: kz[1], kz[3] of the lane whose row differs by 1
};
__device__ inline MomentCoef moment_coef(int lane) {
  const int tap = (lane >> 2) & 15, c = tap & 3, r = tap >> 2;
  MomentCoef m;
  m.kx[0] = keys_coef(c, c);
  m.kx[1] = keys_coef(c, dppi<DPP_ROR4>(c));
  m.kx[2] = keys_coef(c, dppi<DPP_ROR8>(c));
  m.kx[3] = keys_coef(c, dppi<DPP_ROR12>(c));
  const float rf = (float)r;
  const float r2 = exch32(rf);
  m.kz0 = keys_coef(r, r);
  const float kz1 = keys_coef(r, (int)exch16(rf));
  m.kz2 = keys_coef(r, (int)r2);
  const float kz3 = keys_coef(r, (int)exch16(r2));
  m.kz1s = exch16(kz1);
  m.kz3s = exch16(kz3);
  return m;
}

// Adds the tap sums of the moments in acc (summed over the wavefront) to the grid
// copy at cell c: the reduce-scatter leaves each lane one moment; the Keys
// coefficients are applied along x by rotations inside the row and along z by
// exchanges between rows.  acc is consumed.
__device__ inline void flush_moments(float* grid, int c, float (&acc)[16], int lane, int my_off,
                                     const MomentCoef& K) {
  const float m = reduce_scatter16(acc, lane);
  float n = K.kx[0] * m;
  n = fmaf(K.kx[1], dpp<DPP_ROR4>(m), n);
  n = fmaf(K.kx[2], dpp<DPP_ROR8>(m), n);
  n = fmaf(K.kx[3], dpp<DPP_ROR12>(m), n);
  // along z: w = kz0 n + kz1 n(row ^ 1) + kz2 n(row ^ 2) + kz3 n(row ^ 3); the two
  // terms from the neighbouring row are formed there and brought over in one exchange
  const float n2 = exch32(n);
  float w = fmaf(K.kz2, n2, K.kz0 * n);
  w += exch16(fmaf(K.kz3s, n2, K.kz1s * n));
  if ((lane & 3) == 0) lds_add(grid + c + my_off, w);
}

// One element's rays from the wavefront's points: start in grid coordinates, step
// per segment, and the adjoint weight dL/dT * L2 / N of the lane's ray.
struct Ray {
  float u0, v0, du, dv, coef;
  bool live;
};

// Ray point k of every lane: its grid position (clamped to the node range) and cell.
__device__ inline int ray_pos(const Ray& r, int k, float umax, float vmax, int W, float& u,
                              float& v) {
  u = __builtin_amdgcn_fmed3f(fmaf((float)k, r.du, r.u0), 0.f, umax);
  v = __builtin_amdgcn_fmed3f(fmaf((float)k, r.dv, r.v0), 0.f, vmax);
  return (int)v * W + (int)u;
}

// Ray point k of one element in moment form: acc[4 b + a] += c_k g^b f^a, with f and
// g the x and z fractions of the point in its cell and c_k the ray's adjoint weight
// (halved at both ends of the trapezoid).  Every Keys weight is a cubic in its
// fraction, so the tap sums of points in one cell are fixed linear combinations of
// these 16 moments (applied once per cell by flush_moments).  A ray point with
// `in` false adds zeros.
__device__ inline void ray_moments(const Ray& r, int k, int nseg, float u, float v, bool in,
                                   float (&acc)[16]) {
  const float f = __builtin_amdgcn_fractf(u), g = __builtin_amdgcn_fractf(v);  // u, v >= 0
  const float f2 = f * f, f3 = f2 * f;
  float gb = (k == 0 || k == nseg) ? 0.5f * r.coef : r.coef;
  gb = in ? gb : 0.f;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    acc[4 * b] += gb;
    acc[4 * b + 1] = fmaf(gb, f, acc[4 * b + 1]);
    acc[4 * b + 2] = fmaf(gb, f2, acc[4 * b + 2]);
    acc[4 * b + 3] = fmaf(gb, f3, acc[4 * b + 3]);
    if (b < 3) gb *= g;
  }
}

// The ray points of NR rays per lane (elements walked together; `all`: the lanes
// with a live ray), ray point k of every ray at step k.  Moments of ray points in
// one cell accumulate in acc (pending for cell c_acc) until a step leaves that
// cell.  A step whose ray points lie in several cells takes one round per cell,
// the pending cell first when the step has points there: each round adds the
// moments of its cell's points and is flushed, except the last, whose cell stays
// pending.
template <int NR>
__device__ inline void walk_rays(float* grid, Ray (&R)[NR], unsigned long long all, int nseg,
                                 float umax, float vmax, int W, int lane, int my_off,
                                 const MomentCoef& kc) {
  const int lead = __ffsll((long long)all) - 1;
  // An idle ray (zero weight) takes the geometry of the lane's first live ray, or
  // in a lane with none, that of the lead lane's first live ray: every ray point of
  // a step then lies in a cell that a live ray point of the step occupies, and the
  // lead lane's ray 0 stands for its first live ray.
  {
    // plain value selects (a conditional copy of the fields would become a load
    // through a selected pointer and put the rays in scratch memory)
    float fu = R[NR - 1].u0, fv = R[NR - 1].v0, fdu = R[NR - 1].du, fdv = R[NR - 1].dv;
    bool any = R[NR - 1].live;
#pragma unroll
    for (int n = NR - 2; n >= 0; --n) {
      const bool l = R[n].live;
      fu = l ? R[n].u0 : fu;
      fv = l ? R[n].v0 : fv;
      fdu = l ? R[n].du : fdu;
      fdv = l ? R[n].dv : fdv;
      any = any || l;
    }
    const float lu = readlane_f(fu, lead), lv = readlane_f(fv, lead);
    const float ldu = readlane_f(fdu, lead), ldv = readlane_f(fdv, lead);
    fu = any ? fu : lu;
    fv = any ? fv : lv;
    fdu = any ? fdu : ldu;
    fdv = any ? fdv : ldv;
#pragma unroll
    for (int n = 0; n < NR; ++n) {
      const bool l = R[n].live;
      R[n].u0 = l ? R[n].u0 : fu;
      R[n].v0 = l ? R[n].v0 : fv;
      R[n].du = l ? R[n].du : fdu;
      R[n].dv = l ? R[n].dv : fdv;
    }
  }
  // acc is all zeros whenever c_acc is -1.
  float acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  int c_acc = -1;  // wavefront-uniform: the cell of the pending sums in acc (-1: none)
  for (int k = 0; k <= nseg; ++k) {
    float u[NR], v[NR];
    int cell[NR];
#pragma unroll
    for (int n = 0; n < NR; ++n) cell[n] = ray_pos(R[n], k, umax, vmax, W, u[n], v[n]);
    const int c0 = __builtin_amdgcn_readlane(cell[0], lead);
    bool one = true;
#pragma unroll
    for (int n = 0; n < NR; ++n) one = one && cell[n] == c0;
    if (__ballot(!one) == 0ull) {  // the usual case: one cell for the whole wavefront
      if (c0 != c_acc && c_acc >= 0) {
        flush_moments(grid, c_acc, acc, lane, my_off, kc);
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.f;
      }
      c_acc = c0;
#pragma unroll
      for (int n = 0; n < NR; ++n) ray_moments(R[n], k, nseg, u[n], v[n], true, acc);
      continue;
    }
    int cur = c0;
    if (c_acc >= 0) {
      bool has = false;
#pragma unroll
      for (int n = 0; n < NR; ++n) has = has || cell[n] == c_acc;
      if (__ballot(has) != 0ull) {
        cur = c_acc;
      } else {
        flush_moments(grid, c_acc, acc, lane, my_off, kc);
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.f;
      }
    }
    bool left[NR];
#pragma unroll
    for (int n = 0; n < NR; ++n) left[n] = true;
    while (true) {  // every round takes at least one ray point (of the lane cur came from)
      bool rem = false;
#pragma unroll
      for (int n = 0; n < NR; ++n) {
        const bool in = left[n] && cell[n] == cur;
        ray_moments(R[n], k, nseg, u[n], v[n], in, acc);
        left[n] = left[n] && !in;
        rem = rem || left[n];
      }
      const unsigned long long rest = __ballot(rem);
      if (rest == 0ull) break;
      flush_moments(grid, cur, acc, lane, my_off, kc);
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[i] = 0.f;
      int nxt = cell[NR - 1];
#pragma unroll
      for (int n = NR - 2; n >= 0; --n) nxt = left[n] ? cell[n] : nxt;
      cur = __builtin_amdgcn_readlane(nxt, __ffsll((long long)rest) - 1);
    }
    c_acc = cur;
  }
  if (c_acc >= 0) flush_moments(grid, c_acc, acc, lane, my_off, kc);
}

// COPIES grid copies per workgroup: 4 (one private copy per wavefront), or for
// large grids, where four copies would keep the CU below four workgroups, 2 (one
// per pair of wavefronts) or 1 (shared by all four).
template <bool DET, int COPIES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_path_adj(PathArgs A) {
  extern __shared__ float sg[];  // [COPIES][nodes]
  const Geo& g = A.g;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int tile = A.order[blockIdx.x];
  const int4 tr = A.tiles[tile];
  const int W = g.W;
  const int nodes = W * (g.nz + 3);
  for (int i = tid; i < COPIES * nodes; i += 256) sg[i] = 0.f;
  __syncthreads();
  float* grid = sg + ((tid >> 6) * COPIES / 4) * nodes;

  const long long p = (long long)tile * TILE + tid;
  const int2 pr = A.prange[p];
  const float2 pxy = A.ptxy[p];
  const float inv_n = 1.f / (float)g.n_seg;
  const float up = (pxy.x - g.x0) * g.idx, vp = (pxy.y - g.z0) * g.idz;
  const float umax = (float)(g.nx - 1), vmax = (float)(g.nz - 1);
  // tap (r, c) of value index i = 4 r + c; this lane's reduced tap
  const int my_tap = (lane >> 2) & 15;
  const int my_off = (my_tap >> 2) * W + (my_tap & 3);
  const MomentCoef kc = moment_coef(lane);

  // Elements four at a time: the rays of neighbouring elements to the same points
  // run side by side, so at a step their ray points usually share one cell and one
  // reduce covers all four.  Where some of the four have no work in this wavefront
  // (the aperture edges), each pair walks on its own, or its one element with work.
  for (int a = tr.x; a <= tr.y; a += 4) {  // wavefront-uniform loop
    Ray R[4];
    unsigned long long lm[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int e = a + n;
      const bool act = e <= tr.y && e >= pr.x && e <= pr.y;
      float gbar = 0.f;
      if (act) {
        gbar = A.gT[(long long)e * g.P + p];  // receive role
        if (DET) {  // the transmit-role slabs in receive-block order
          const float* q = A.gtp + A.tbase[tile] + (long long)(e - tr.x) * TILE + tid;
          const long long slab = (long long)(tr.y - tr.x + 1) * TILE;
          for (int jb = tr.z; jb <= tr.w; ++jb) gbar += q[(long long)(jb - tr.z) * slab];
        } else {
          gbar += A.gT2[(long long)e * g.P + p];
        }
      }
      R[n].live = act && gbar != 0.f;
      lm[n] = __ballot(R[n].live);
      R[n].coef = 0.f;
      R[n].u0 = R[n].v0 = R[n].du = R[n].dv = 0.f;
      if (lm[n] != 0ull) {
        const float2 ruv = A.ray_uv[(long long)e * g.P + p];
        if (R[n].live) R[n].coef = gbar * A.ray_l2[(long long)e * g.P + p] * inv_n;
        R[n].u0 = ruv.x;
        R[n].v0 = ruv.y;
        R[n].du = (up - ruv.x) * inv_n;
        R[n].dv = (vp - ruv.y) * inv_n;
      }
    }
    const unsigned long long all = lm[0] | lm[1] | lm[2] | lm[3];
    if (all == 0ull) continue;
    if (lm[0] != 0ull && lm[1] != 0ull && lm[2] != 0ull && lm[3] != 0ull) {
      walk_rays<4>(grid, R, all, g.n_seg, umax, vmax, W, lane, my_off, kc);
      continue;
    }
    // some element of the four has no work in this wavefront: pairs and singles
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const unsigned long long m0 = lm[2 * h], m1 = lm[2 * h + 1];
      if ((m0 | m1) == 0ull) continue;
      if (m0 == 0ull || m1 == 0ull) {  // one element with work
        const bool s0 = m0 != 0ull;
        Ray R1[1];
        R1[0].u0 = s0 ? R[2 * h].u0 : R[2 * h + 1].u0;
        R1[0].v0 = s0 ? R[2 * h].v0 : R[2 * h + 1].v0;
        R1[0].du = s0 ? R[2 * h].du : R[2 * h + 1].du;
        R1[0].dv = s0 ? R[2 * h].dv : R[2 * h + 1].dv;
        R1[0].coef = s0 ? R[2 * h].coef : R[2 * h + 1].coef;
        R1[0].live = s0 ? R[2 * h].live : R[2 * h + 1].live;
        walk_rays<1>(grid, R1, m0 | m1, g.n_seg, umax, vmax, W, lane, my_off, kc);
        continue;
      }
      Ray R2[2] = {R[2 * h], R[2 * h + 1]};
      walk_rays<2>(grid, R2, m0 | m1, g.n_seg, umax, vmax, W, lane, my_off, kc);
    }
  }
  __syncthreads();
  // per-workgroup partial grid (plain stores); summed in fixed order by k_path_reduce
  float* part = A.gpart + (long long)blockIdx.x * nodes;
  for (int n = tid; n < nodes; n += 256)
    part[n] = COPIES == 1   ? sg[n]
              : COPIES == 2 ? sg[n] + sg[nodes + n]
                            : (sg[n] + sg[nodes + n]) + (sg[2 * nodes + n] + sg[3 * nodes + n]);
}

// gpad[n] = sum over workgroups of their partial grids, in a fixed order
// (deterministic), in two passes: k_path_chunk sums each chunk of PCHUNK
// consecutive partial grids into the first grid of the chunk (every element is
// read and then overwritten by the same thread), k_path_reduce sums the chunks.
constexpr int PCHUNK = 32;

__global__ __launch_bounds__(256) void k_path_chunk(float* __restrict__ gpart, int n_wg, int nodes) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  const int w0 = blockIdx.y * PCHUNK;
  if (n >= nodes) return;
  const int w1 = min(w0 + PCHUNK, n_wg);
  float v[PCHUNK];
#pragma unroll
  for (int k = 0; k < PCHUNK; ++k) v[k] = (w0 + k < w1) ? gpart[(long long)(w0 + k) * nodes + n] : 0.f;
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < PCHUNK; ++k) s += v[k];
  gpart[(long long)w0 * nodes + n] = s;
}

__global__ __launch_bounds__(256) void k_path_reduce(const float* __restrict__ gpart, int n_wg,
                                                     int nodes, float* __restrict__ gpad) {
  const int n = blockIdx.x * 64 + (threadIdx.x & 63);
  const int lane_grp = threadIdx.x >> 6;  // 4 groups stride over the chunks
  const int n_chunk = (n_wg + PCHUNK - 1) / PCHUNK;
  __shared__ float red[4][64];
  float s = 0.f;
  if (n < nodes)
    for (int c = lane_grp; c < n_chunk; c += 4) s += gpart[(long long)c * PCHUNK * nodes + n];
  red[lane_grp][threadIdx.x & 63] = s;
  __syncthreads();
  if (lane_grp == 0 && n < nodes)
    gpad[n] = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

__global__ __launch_bounds__(256) void k_zero(float* __restrict__ x, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = 0.f;
}

}  // namespace

hipError_t launch_sum_grids(af_ctx* c, float* parts, int n, float* out) {
  const int nodes = (c->nx + 3) * (c->nz + 3);
  const int n_chunk = (n + PCHUNK - 1) / PCHUNK;
  hipLaunchKernelGGL(k_path_chunk, dim3((nodes + 255) / 256, n_chunk), dim3(256), 0, c->stream,
                     parts, n, nodes);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_path_reduce, dim3((nodes + 63) / 64), dim3(256), 0, c->stream, parts, n,
                     nodes, out);
  return hipGetLastError();
}

hipError_t launch_path_adj(af_ctx* c, float* out) {
  const int nodes = (c->nx + 3) * (c->nz + 3);
  if (c->v.n_order == 0) {
    hipLaunchKernelGGL(k_zero, dim3((nodes + 255) / 256), dim3(256), 0, c->stream, out,
                       (long long)nodes);
    return hipGetLastError();
  }
  PathArgs A{};
  A.g = c->geo();
  A.ray_uv = c->d_ray_uv.as<float2>();
  A.ray_l2 = c->d_ray_l2.as<float>();
  A.ptxy = c->v.ptxy;
  A.prange = c->v.prange;
  A.tiles = c->v.tiles;
  A.order = c->v.order;
  A.gT = c->d_gT.as<float>();
  A.gT2 = c->d_gT.as<float>() + (size_t)c->N * c->v.P;
  A.gtp = c->d_gtp.as<float>();
  A.tbase = c->v.tbase;
  A.gpart = c->d_gpart.as<float>();
  // the most copies (4, 2 or 1) of which four workgroups fit the CU's 160 KB of LDS
  // (deterministic mode keeps four private copies)
  const size_t per = sizeof(float) * (size_t)nodes * 4;  // one copy in four workgroups
  const int copies = c->det ? 4 : per * 4 <= 160 * 1024 ? 4 : per * 2 <= 160 * 1024 ? 2 : 1;
  const size_t lds = sizeof(float) * (size_t)nodes * copies;
  const dim3 grid(c->v.n_order), block(256);
  if (c->det)
    hipLaunchKernelGGL((k_path_adj<true, 4>), grid, block, lds, c->stream, A);
  else if (copies == 4)
    hipLaunchKernelGGL((k_path_adj<false, 4>), grid, block, lds, c->stream, A);
  else if (copies == 2)
    hipLaunchKernelGGL((k_path_adj<false, 2>), grid, block, lds, c->stream, A);
  else
    hipLaunchKernelGGL((k_path_adj<false, 1>), grid, block, lds, c->stream, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_grids(c, c->d_gpart.as<float>(), c->v.n_order, out);
}

}  // namespace af
