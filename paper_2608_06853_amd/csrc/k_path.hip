// Adjoint of the path integral: dL/ds[node] += sum over rays and ray points of
// dL/dT * L2 * w_k * (bicubic weight of the node at r_k) / N.  Refraction points
// and c_med are held constant (they follow the global mean speed); each ray's
// start and medium leg L2 are read from the table kernel of the same slowness.
//
// A workgroup takes one tile of points and every active element of it; a
// wavefront walks the rays from the elements to its 64 points in lock step.  The
// rays are nearly parallel, so at a given step the lanes usually sit in one grid
// cell.  Consecutive such steps add the 16 moments c g^b f^a of their ray points
// (f, g: the fractions in the cell) into registers; when the cell changes, the
// moments are summed across the wavefront with a reduce-scatter, turned into the
// 16 tap sums by the Keys coefficients (lane rotations and row exchanges), and 16
// lanes add them to an LDS copy of the padded grid with LDS float atomics.  Lanes
// spread over two neighbouring cells are summed as one window of 4 x 5 or 5 x 4
// nodes; lanes spread wider are handled one cell at a time.  The rays of four
// neighbouring elements are walked together and summed by the same reduce whenever
// their cells allow it (else by pairs).  The copies are summed into one partial
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
template <int CTRL>
__device__ inline float dpp(float x) {
  return __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(x), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ inline int dppi(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xf, 0xf, false);
}
constexpr int DPP_ROR8 = 0x128, DPP_HALF_MIRROR = 0x141, DPP_XOR2 = 0x4e, DPP_XOR1 = 0xb1;
constexpr int DPP_ROR12 = 0x12c, DPP_ROR4 = 0x124, DPP_ROR2 = 0x122, DPP_ROR1 = 0x121;

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
  float kx[4], kz[4];
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
  m.kz[0] = keys_coef(r, r);
  m.kz[1] = keys_coef(r, (int)exch16(rf));
  m.kz[2] = keys_coef(r, (int)r2);
  m.kz[3] = keys_coef(r, (int)exch16(r2));
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
  const float n2 = exch32(n);
  float w = K.kz[0] * n;
  w = fmaf(K.kz[1], exch16(n), w);
  w = fmaf(K.kz[2], n2, w);
  w = fmaf(K.kz[3], exch16(n2), w);
  if ((lane & 3) == 0) lds_add(grid + c + my_off, w);
}

// Sum over the wavefront of v[r], r = 0..3: every lane returns the sum of
// v[l >> 4].  The half-wave swaps leave row r (16 lanes) holding value r summed
// over four lanes; rotations by 8, 4, 2 and 1 inside the row finish the sum.
__device__ inline float reduce_scatter4(float v[4]) {
  swap32(v[0], v[2]);  // lower half: value 0; upper half: value 2
  v[0] += v[2];
  swap32(v[1], v[3]);  // lower half: value 1; upper half: value 3
  v[1] += v[3];
  swap16(v[0], v[1]);  // rows 0, 2: v[0] of both rows; rows 1, 3: v[1] of both rows
  float h = v[0] + v[1];
  h += dpp<DPP_ROR8>(h);
  h += dpp<DPP_ROR4>(h);
  h += dpp<DPP_ROR2>(h);
  h += dpp<DPP_ROR1>(h);
  return h;
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

// The two weight vectors of ray point k at (u, v) whose outer product az x wx gives
// the 16 tap weights (trapezoid end weights folded into az).
__device__ inline void ray_weights(const Ray& r, int k, int nseg, float u, float v, float az[4],
                                   float wx[4]) {
  keys_weights(__builtin_amdgcn_fractf(u), wx[0], wx[1], wx[2], wx[3]);  // u, v >= 0: u - j0
  const float ck = (k == 0 || k == nseg) ? 0.5f * r.coef : r.coef;
  keys_weights_scaled(__builtin_amdgcn_fractf(v), ck, az[0], az[1], az[2], az[3]);
}

// Ray point k of every lane: returns its cell and the two weight vectors.
__device__ inline int ray_point(const Ray& r, int k, int nseg, float umax, float vmax, int W,
                                float az[4], float wx[4]) {
  float u, v;
  const int cell = ray_pos(r, k, umax, vmax, W, u, v);
  ray_weights(r, k, nseg, u, v, az, wx);
  return cell;
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

// NR ray points per lane whose cells lie in two neighbouring cells, cb and cb + 1
// (horizontal) or cb and cb + W (vertical): every ray point shifts its four weights
// along that axis into a window of five nodes (by one place if it is in the second
// cell), so the union of the taps is a 4 x 5 (or 5 x 4) block at cb.  Its first 16
// nodes are summed by the 16-value reduce-scatter, the last row or column of four by
// the 4-value one.  (Cells never exceed node nx - 1 or nz - 1, so the window's
// fifth column or row stays inside the padded grid.)
template <bool HORIZONTAL, int NR>
__device__ inline void scatter_window(float* grid, int cb, int W, const float (&a)[NR][4],
                                      const float (&b)[NR][4], const bool (&shift)[NR], int lane,
                                      int my_off) {
  float v16[16], v4[4];
#pragma unroll
  for (int i = 0; i < 16; ++i) v16[i] = 0.f;
#pragma unroll
  for (int q = 0; q < 4; ++q) v4[q] = 0.f;
#pragma unroll
  for (int n = 0; n < NR; ++n) {
    if (HORIZONTAL) {
      float bs[5];
      bs[0] = shift[n] ? 0.f : b[n][0];
#pragma unroll
      for (int c = 1; c < 4; ++c) bs[c] = shift[n] ? b[n][c - 1] : b[n][c];
      bs[4] = shift[n] ? b[n][3] : 0.f;
#pragma unroll
      for (int i = 0; i < 16; ++i) v16[i] = fmaf(a[n][i >> 2], bs[i & 3], v16[i]);
#pragma unroll
      for (int r = 0; r < 4; ++r) v4[r] = fmaf(a[n][r], bs[4], v4[r]);
    } else {
      float as[5];
      as[0] = shift[n] ? 0.f : a[n][0];
#pragma unroll
      for (int r = 1; r < 4; ++r) as[r] = shift[n] ? a[n][r - 1] : a[n][r];
      as[4] = shift[n] ? a[n][3] : 0.f;
#pragma unroll
      for (int i = 0; i < 16; ++i) v16[i] = fmaf(as[i >> 2], b[n][i & 3], v16[i]);
#pragma unroll
      for (int c = 0; c < 4; ++c) v4[c] = fmaf(as[4], b[n][c], v4[c]);
    }
  }
  const float sum16 = reduce_scatter16(v16, lane);
  if ((lane & 3) == 0) lds_add(grid + cb + my_off, sum16);
  const float sum4 = reduce_scatter4(v4);
  // node 4 of row (lane >> 4), or node (lane >> 4) of row 4
  const int off4 = HORIZONTAL ? (lane >> 4) * W + 4 : 4 * W + (lane >> 4);
  if ((lane & 15) == 0) lds_add(grid + cb + off4, sum4);
}

// Adds the tap weights of NR ray points per lane (cells in `cell`, idle lanes
// already moved to c0 with zero weights) when the union of their cells is the one
// cell c0 or two neighbouring cells; returns false, writing nothing, otherwise.
template <int NR>
__device__ inline bool scatter_union(float* grid, int c0, int W, const int (&cell)[NR],
                                     const float (&az)[NR][4], const float (&wx)[NR][4], int lane,
                                     int my_off) {
  bool one = true;
#pragma unroll
  for (int n = 0; n < NR; ++n) one = one && cell[n] == c0;
  if (__ballot(!one) == 0ull) {  // the usual case: one cell for the whole wavefront
    float val[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      val[i] = az[0][i >> 2] * wx[0][i & 3];
#pragma unroll
      for (int n = 1; n < NR; ++n) val[i] = fmaf(az[n][i >> 2], wx[n][i & 3], val[i]);
    }
    const float sum = reduce_scatter16(val, lane);
    if ((lane & 3) == 0) lds_add(grid + c0 + my_off, sum);
    return true;
  }
  // the other cell, relative to c0: +1, -1, +W or -W for every lane (0 if none)
  int d = 0;
#pragma unroll
  for (int n = 0; n < NR; ++n) d = cell[n] != c0 ? cell[n] - c0 : d;
  const int dd = __builtin_amdgcn_readlane(d, __ffsll((long long)__ballot(d != 0)) - 1);
  bool same = true;
#pragma unroll
  for (int n = 0; n < NR; ++n) same = same && (cell[n] == c0 || cell[n] - c0 == dd);
  if (__ballot(!same) != 0ull || (dd != 1 && dd != -1 && dd != W && dd != -W)) return false;
  bool shift[NR];
  const bool h = dd == 1, hl = dd == -1, v = dd == W;
  if (h) {
#pragma unroll
    for (int n = 0; n < NR; ++n) shift[n] = cell[n] != c0;
    scatter_window<true, NR>(grid, c0, W, az, wx, shift, lane, my_off);
    return true;
  }
  if (hl) {
#pragma unroll
    for (int n = 0; n < NR; ++n) shift[n] = cell[n] == c0;
    scatter_window<true, NR>(grid, c0 - 1, W, az, wx, shift, lane, my_off);
    return true;
  }
  if (v) {
#pragma unroll
    for (int n = 0; n < NR; ++n) shift[n] = cell[n] != c0;
    scatter_window<false, NR>(grid, c0, W, az, wx, shift, lane, my_off);
    return true;
  }
#pragma unroll
  for (int n = 0; n < NR; ++n) shift[n] = cell[n] == c0;
  scatter_window<false, NR>(grid, c0 - W, W, az, wx, shift, lane, my_off);
  return true;
}

// One ray point per lane spread over more cells: one masked reduce round per
// distinct cell (idle lanes already moved to c0 with zero weights).
__device__ inline void scatter_rounds(float* grid, int c0, int cell, const float (&az)[4],
                                      const float (&wx)[4], int lane, int my_off) {
  float val[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) val[i] = az[i >> 2] * wx[i & 3];
  bool done = false;
  int ccur = c0;
  while (true) {
    const bool in = !done && cell == ccur;
    float vv[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) vv[i] = in ? val[i] : 0.f;
    const float sum = reduce_scatter16(vv, lane);
    if ((lane & 3) == 0) lds_add(grid + ccur + my_off, sum);
    done = done || in;
    const unsigned long long rest = __ballot(!done);
    if (rest == 0ull) break;
    ccur = __builtin_amdgcn_readlane(cell, __ffsll((long long)rest) - 1);
  }
}

// One ray point per lane, any spread.
__device__ inline void scatter_one(float* grid, int cell, bool live, int lead, int W,
                                   const float (&az)[4], const float (&wx)[4], int lane,
                                   int my_off) {
  const int c0 = __builtin_amdgcn_readlane(cell, lead);
  const int c[1] = {live ? cell : c0};  // idle lanes (zero weights) join the leader's cell
  const float a1[1][4] = {{az[0], az[1], az[2], az[3]}};
  const float b1[1][4] = {{wx[0], wx[1], wx[2], wx[3]}};
  if (!scatter_union<1>(grid, c0, W, c, a1, b1, lane, my_off))
    scatter_rounds(grid, c0, c[0], az, wx, lane, my_off);
}

// Ray point k of the rays of two elements (either may be idle in a lane): one
// reduce when their cells allow it, else each element on its own.
__device__ inline void scatter_pair(float* grid, const int (&cell)[2], const bool (&live)[2],
                                    int lead, int lead0, int lead1, int W,
                                    const float (&az)[2][4], const float (&wx)[2][4], int lane,
                                    int my_off) {
  const int c0 = __builtin_amdgcn_readlane(live[0] ? cell[0] : cell[1], lead);
  const int cu[2] = {live[0] ? cell[0] : c0, live[1] ? cell[1] : c0};
  if (scatter_union<2>(grid, c0, W, cu, az, wx, lane, my_off)) return;
  // the two ray points of a lane lie wider apart: each element on its own
  scatter_one(grid, cell[0], live[0], lead0, W, az[0], wx[0], lane, my_off);
  scatter_one(grid, cell[1], live[1], lead1, W, az[1], wx[1], lane, my_off);
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
  // run side by side, so at a step their ray points usually share one cell (or two
  // neighbouring cells) and one reduce covers all four; otherwise the step falls
  // back to the two pairs, and a pair to its single elements.
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
    int leads[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) leads[n] = __ffsll((long long)lm[n]) - 1;
    if (lm[0] != 0ull && lm[1] != 0ull && lm[2] != 0ull && lm[3] != 0ull) {
      const int lead = __ffsll((long long)all) - 1;
      // An idle ray (zero weight) takes the geometry of the lane's first live ray,
      // or in a lane with none, that of the lead lane's first live ray: every ray
      // point of a step then lies in a cell that a live ray point of the step
      // occupies, and the lead lane's ray 0 stands for its first live ray.
      {
        float fu = R[3].u0, fv = R[3].v0, fdu = R[3].du, fdv = R[3].dv;
#pragma unroll
        for (int n = 2; n >= 0; --n)
          if (R[n].live) {
            fu = R[n].u0;
            fv = R[n].v0;
            fdu = R[n].du;
            fdv = R[n].dv;
          }
        const float lu = readlane_f(fu, lead), lv = readlane_f(fv, lead);
        const float ldu = readlane_f(fdu, lead), ldv = readlane_f(fdv, lead);
        if (!(R[0].live || R[1].live || R[2].live || R[3].live)) {
          fu = lu;
          fv = lv;
          fdu = ldu;
          fdv = ldv;
        }
#pragma unroll
        for (int n = 0; n < 4; ++n)
          if (!R[n].live) {
            R[n].u0 = fu;
            R[n].v0 = fv;
            R[n].du = fdu;
            R[n].dv = fdv;
          }
      }
      // Moments of ray points in one cell accumulate in acc (pending for cell c_acc)
      // until a step leaves that cell.  A step whose ray points lie in several cells
      // takes one round per cell, the pending cell first when the step has points
      // there: each round adds the moments of its cell's points and is flushed,
      // except the last, whose cell stays pending.
      // acc is all zeros whenever c_acc is -1.
      float acc[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[i] = 0.f;
      int c_acc = -1;  // wavefront-uniform: the cell of the pending sums in acc (-1: none)
      for (int k = 0; k <= g.n_seg; ++k) {
        float u[4], v[4];
        int cell[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) cell[n] = ray_pos(R[n], k, umax, vmax, W, u[n], v[n]);
        const int c0 = __builtin_amdgcn_readlane(cell[0], lead);
        bool one = true;
#pragma unroll
        for (int n = 0; n < 4; ++n) one = one && cell[n] == c0;
        if (__ballot(!one) == 0ull) {  // the usual case: one cell for the whole wavefront
          if (c0 != c_acc && c_acc >= 0) {
            flush_moments(grid, c_acc, acc, lane, my_off, kc);
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[i] = 0.f;
          }
          c_acc = c0;
#pragma unroll
          for (int n = 0; n < 4; ++n) ray_moments(R[n], k, g.n_seg, u[n], v[n], true, acc);
          continue;
        }
        int cur = c0;
        if (c_acc >= 0) {
          bool has = false;
#pragma unroll
          for (int n = 0; n < 4; ++n) has = has || cell[n] == c_acc;
          if (__ballot(has) != 0ull) {
            cur = c_acc;
          } else {
            flush_moments(grid, c_acc, acc, lane, my_off, kc);
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[i] = 0.f;
          }
        }
        bool left[4] = {true, true, true, true};
        while (true) {  // every round takes at least one ray point (of the lane cur came from)
#pragma unroll
          for (int n = 0; n < 4; ++n) {
            const bool in = left[n] && cell[n] == cur;
            ray_moments(R[n], k, g.n_seg, u[n], v[n], in, acc);
            left[n] = left[n] && !in;
          }
          const unsigned long long rest = __ballot(left[0] || left[1] || left[2] || left[3]);
          if (rest == 0ull) break;
          flush_moments(grid, cur, acc, lane, my_off, kc);
#pragma unroll
          for (int i = 0; i < 16; ++i) acc[i] = 0.f;
          const int nxt = left[0] ? cell[0] : left[1] ? cell[1] : left[2] ? cell[2] : cell[3];
          cur = __builtin_amdgcn_readlane(nxt, __ffsll((long long)rest) - 1);
        }
        c_acc = cur;
      }
      if (c_acc >= 0) flush_moments(grid, c_acc, acc, lane, my_off, kc);
      continue;
    }
    // some element of the four has no work in this wavefront: pairs and singles
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const unsigned long long m0 = lm[2 * h], m1 = lm[2 * h + 1];
      if ((m0 | m1) == 0ull) continue;
      if (m0 == 0ull || m1 == 0ull) {  // one element with work
        const Ray& r = m0 != 0ull ? R[2 * h] : R[2 * h + 1];
        const int lead = __ffsll((long long)(m0 | m1)) - 1;
        for (int k = 0; k <= g.n_seg; ++k) {
          float az[4], wx[4];
          const int cell = ray_point(r, k, g.n_seg, umax, vmax, W, az, wx);
          scatter_one(grid, cell, r.live, lead, W, az, wx, lane, my_off);
        }
        continue;
      }
      const int lead = __ffsll((long long)(m0 | m1)) - 1;
      const bool l2[2] = {R[2 * h].live, R[2 * h + 1].live};
      for (int k = 0; k <= g.n_seg; ++k) {
        float az[2][4], wx[2][4];
        int cell[2];
#pragma unroll
        for (int n = 0; n < 2; ++n)
          cell[n] = ray_point(R[2 * h + n], k, g.n_seg, umax, vmax, W, az[n], wx[n]);
        scatter_pair(grid, cell, l2, lead, leads[2 * h], leads[2 * h + 1], W, az, wx, lane, my_off);
      }
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
