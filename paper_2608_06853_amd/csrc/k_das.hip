// Synthetic-aperture delay-and-sum with phase rotation (Eq. 5) over block pairs,
// and its adjoint with respect to the one-way travel times.
//
// A workgroup owns one tile of 256 spatially compact points (one point per
// thread) and loops only over the elements that are active (apodisation,
// Eq. 4) for some point of the tile.  Each sample is a linear interpolation of
// two adjacent IQ samples of channel (t, r) at u = u_t + u_r, rotated by the
// product of the two per-element phasors from the travel-time table.
#include "af_internal.h"

namespace af {
namespace {

struct Rx {
  int ui;
  float uf;
  float2 e;
};

// Receive-role table entry; elements outside the tile's range act as masked
// entries (sample 0, zero phasor), exactly like the masked entries of the table.
__device__ inline Rx load_rx(const TabEntry* __restrict__ tab, long long P, long long p, int r,
                             int LO, int HI) {
  Rx x;
  if (r >= LO && r <= HI) {
    const TabEntry te = tab[(long long)r * P + p];
    x.ui = te.ui;
    x.uf = te.uf;
    x.e = make_float2(te.er, te.ei);
  } else {
    x.ui = 0;
    x.uf = 0.f;
    x.e = make_float2(0.f, 0.f);
  }
  return x;
}

// Sample index of channel (t, r) with its record check: returns false when u lies
// outside [0, ns-1] (u = ns-1 exactly reads the last sample).
__device__ inline bool sample_pos(int ui_t, float uf_t, int ui_r, float uf_r, int ns, int& k,
                                  float& f) {
  int kk = ui_t + ui_r;
  float fsum = uf_t + uf_r;
  const int carry = fsum >= 1.f ? 1 : 0;
  kk += carry;
  f = fsum - (float)carry;
  if (kk == ns - 1 && f == 0.f) {
    kk = ns - 2;
    f = 1.f;
  }
  k = kk;
  return (unsigned)kk <= (unsigned)(ns - 2);
}

__device__ inline int wave_min(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline int wave_max(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// The S gathers of one transmit element t for this lane's point.  With CHECK
// the record bounds are tested per sample (a sample outside the record reads
// the first two samples of its channel and is zeroed); without, the caller has
// shown for the whole wavefront that every sample lies strictly inside the
// record.  Masked entries carry a zero phasor and contribute nothing either way.
template <int S, bool CHECK, bool SKIP = false>
__device__ inline void gather(const float2* __restrict__ base, int ns, const TabEntry& et,
                              const Rx (&rx)[S], float2 (&a0)[S], float2 (&a1)[S], float (&fr)[S],
                              bool (&ok)[S]) {
  const bool t_on = et.er != 0.f || et.ei != 0.f;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    int kk;
    if (CHECK) {
      ok[k] = sample_pos(et.ui, et.uf, rx[k].ui, rx[k].uf, ns, kk, fr[k]);
      if (!ok[k]) kk = 0;
    } else {
      // fsum lies in [0, 2): its integer part is the carry, its fraction the weight
      const float fsum = et.uf + rx[k].uf;
      kk = et.ui + rx[k].ui + (int)fsum;
      fr[k] = __builtin_amdgcn_fractf(fsum);
      ok[k] = true;
    }
    const float2* q = base + (unsigned)(k * ns + kk);
    if (SKIP) {  // a lane whose sample is apodised out (zero phasor) loads nothing
      float2 v0 = make_float2(0.f, 0.f), v1 = v0;
      if (t_on && (rx[k].e.x != 0.f || rx[k].e.y != 0.f)) {
        v0 = q[0];
        v1 = q[1];
      }
      a0[k] = v0;
      a1[k] = v1;
    } else {
      a0[k] = q[0];
      a1[k] = q[1];
    }
  }
}

// Wavefront-uniform choice of the unchecked path for transmit element t: every
// lane's samples u = u_t + u_r (r in the block) satisfy 0 <= u < ns - 1.
__device__ inline bool interior(const TabEntry& et, int rmin, int rmax, int ns) {
  const bool in = et.ui + rmin >= 0 && et.ui + rmax + 1 <= ns - 2;
  return __ballot(!in) == 0ull;
}

// Span of the sample index sums of this lane's active receive entries (nonzero
// phasor); lo > hi when none is active.
struct RxSpan {
  int lo, hi;
};
template <int S>
__device__ inline RxSpan rx_span(const Rx (&rx)[S]) {
  RxSpan sp{1 << 29, -(1 << 29)};
#pragma unroll
  for (int k = 0; k < S; ++k)
    if (rx[k].e.x != 0.f || rx[k].e.y != 0.f) {
      sp.lo = min(sp.lo, rx[k].ui);
      sp.hi = max(sp.hi, rx[k].ui);
    }
  return sp;
}

// Wavefront-uniform: no lane has a sample of transmit element t inside the
// record.  A sample reads index ui_t + ui_r + carry (carry 0 or 1) and counts
// only for an index in [0, ns - 1], so a lane contributes nothing when its
// transmit entry is masked or every ui_t + ui_r lies above ns - 1 or below -1.
// (Taken only for wavefronts that are not entirely inside the record.)
__device__ inline bool wave_silent(const TabEntry& et, RxSpan sp, int ns) {
  const bool live = (et.er != 0.f || et.ei != 0.f) && et.ui + sp.hi + 1 >= 0 &&
                    et.ui + sp.lo <= ns - 1;
  return __ballot(live) == 0ull;
}
// The same test with the span formed on the spot (for kernels at their register
// limit, where keeping the span across the transmit loop would spill).
template <int S>
__device__ inline bool wave_silent(const TabEntry& et, const Rx (&rx)[S], int ns) {
  return wave_silent(et, rx_span<S>(rx), ns);
}

template <int S, bool CHECK, bool SKIP>
__device__ inline void das_fwd_t(const float2* __restrict__ base, int ns, const TabEntry& et,
                                 const Rx (&rx)[S], float2& acc) {
  float2 a0[S], a1[S];
  float fr[S];
  bool ok[S];
  gather<S, CHECK, SKIP>(base, ns, et, rx, a0, a1, fr, ok);
  float ax = 0.f, ay = 0.f;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const float f = fr[k];
    float vx = fmaf(f, a1[k].x - a0[k].x, a0[k].x);
    float vy = fmaf(f, a1[k].y - a0[k].y, a0[k].y);
    if (CHECK) {
      vx = ok[k] ? vx : 0.f;
      vy = ok[k] ? vy : 0.f;
    }
    ax = fmaf(vx, rx[k].e.x, fmaf(-vy, rx[k].e.y, ax));
    ay = fmaf(vx, rx[k].e.y, fmaf(vy, rx[k].e.x, ay));
  }
  acc.x = fmaf(ax, et.er, fmaf(-ay, et.ei, acc.x));
  acc.y = fmaf(ax, et.ei, fmaf(ay, et.er, acc.y));
}

// Active transmit range of this wavefront's points within the tile range, and
// whether any of them has an active element in receive block jb.
struct WaveRange {
  int lo, hi;
  bool rx_active;
};
__device__ inline WaveRange wave_range(const int2* __restrict__ prange, long long p, int4 tr, int jb,
                                       int S) {
  const int2 pr = prange[p];
  const bool act = pr.x <= pr.y;
  WaveRange w;
  // the same in every lane: read from lane 0 so that loops over the range, and
  // the addresses formed from it, live in scalar registers
  w.lo = __builtin_amdgcn_readfirstlane(max(wave_min(act ? pr.x : 1 << 30), tr.x));
  w.hi = __builtin_amdgcn_readfirstlane(min(wave_max(act ? pr.y : -1), tr.y));
  const bool hit = act && pr.x <= jb * S + S - 1 && pr.y >= jb * S;
  w.rx_active = __ballot(hit) != 0ull;
  return w;
}

// One workgroup per (tile, receive block jb): the block images B^blk[ib][jb] of
// the tile's points for every transmit block ib of the tile.  A wavefront skips
// the transmit elements outside its points' active ranges (their samples are all
// masked) and still writes its zero images.
template <int S>
__global__ __launch_bounds__(256) void k_das_fwd(DasArgs A) {
  const Geo& g = A.g;
  const int2 w = A.work[blockIdx.x];
  const int tile = w.x, jb = w.y;
  if (tile < 0) return;  // padding item of a shorter XCD queue
  const int4 tr = A.tiles[tile];
  const long long P = g.P;
  const long long p = (long long)tile * TILE + threadIdx.x;
  const int N = g.n_elem, ns = g.ns;

  Rx rx[S];
  int rmin = 0, rmax = 0;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    rx[k] = load_rx(A.tab, P, p, jb * S + k, tr.x, tr.y);
    rmin = min(rmin, rx[k].ui);
    rmax = max(rmax, rx[k].ui);
  }
  const WaveRange wr = wave_range(A.prange, p, tr, jb, S);
  const int tlo = wr.rx_active ? wr.lo : tr.y + 1, thi = wr.rx_active ? wr.hi : tr.x - 1;
  const RxSpan sp = rx_span<S>(rx);
  // every lane's receive entries all active: then only a masked transmit entry
  // leaves a lane's samples out (the gathers skip apodised samples only where some are)
  bool rx_on = true;
#pragma unroll
  for (int k = 0; k < S; ++k) rx_on = rx_on && (rx[k].e.x != 0.f || rx[k].e.y != 0.f);
  const bool rx_full = __ballot(!rx_on) == 0ull;

  for (int ib = tr.z; ib <= tr.w; ++ib) {
    float2 acc = make_float2(0.f, 0.f);
    const int t0 = max(ib * S, tlo), t1 = min(ib * S + S - 1, thi);
    if (t0 <= t1) {
      TabEntry et = A.tab[(long long)t0 * P + p];
      for (int t = t0; t <= t1; ++t) {
        const TabEntry en = A.tab[(long long)min(t + 1, t1) * P + p];
        const float2* __restrict__ base = A.iq + ((long long)t * N + (long long)jb * S) * ns;
        if (interior(et, rmin, rmax, ns)) {
          if (rx_full && __ballot(et.er == 0.f && et.ei == 0.f) == 0ull)
            das_fwd_t<S, false, false>(base, ns, et, rx, acc);
          else
            das_fwd_t<S, false, true>(base, ns, et, rx, acc);
        } else if (!wave_silent(et, sp, ns)) {
          das_fwd_t<S, true, true>(base, ns, et, rx, acc);
        }
        et = en;
      }
    }
    A.bblk[((long long)ib * g.nblk + jb) * P + p] = acc;
  }
}

template <int S, bool CHECK>
__device__ inline void das_adj_t(const float2* __restrict__ base, int ns, const TabEntry& et,
                                 const Rx (&rx)[S], float qx, float qy, float fsf, float om,
                                 float (&grx)[S], float& gtx) {
  float2 a0[S], a1[S];
  float fr[S];
  bool ok[S];
  gather<S, CHECK>(base, ns, et, rx, a0, a1, fr, ok);
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const float f = fr[k];
    // D = Re(Q E_r (fs v' + j om v)) = fs Re(P v') - om Im(P v) with P = Q E_r,
    // where v' = a1 - a0 is the sample slope and v the interpolated sample
    const float px = fmaf(qx, rx[k].e.x, -qy * rx[k].e.y);
    const float py = fmaf(qx, rx[k].e.y, qy * rx[k].e.x);
    const float dx = a1[k].x - a0[k].x, dy = a1[k].y - a0[k].y;
    const float vx = fmaf(f, dx, a0[k].x), vy = fmaf(f, dy, a0[k].y);
    const float re_pd = fmaf(px, dx, -py * dy);
    const float im_pv = fmaf(px, vy, py * vx);
    float D = fmaf(fsf, re_pd, -om * im_pv);
    if (CHECK) D = ok[k] ? D : 0.f;
    gtx += D;
    grx[k] += D;
  }
}

// dL/dT[a][p]: for each sample, D = Re(conj(G) (v' + j w v) E_t E_r) feeds the
// transmit element t and the receive element r.  One workgroup per (tile,
// receive block) as in the forward: the receive-role sums of its S elements are
// complete and written directly; the transmit-role sums of every t of the tile
// are partial (over the S receive elements of this block).  By default they are
// added into gT2 with global float atomics (merged in L2; the order of the adds,
// and so the last bits of the sum, vary from run to run).  With DET they go with
// plain stores into this item's own slab, which the path adjoint adds up in
// receive-block order: the gradient is then the same bit for bit on every run,
// at the cost of writing and reading every slab through HBM.
// The register budget is capped at 128 so that 4 wavefronts fit per SIMD; without
// the cap the compiler lands at 131 registers and loses one wavefront per SIMD.
template <int S, bool DET>
__global__ __launch_bounds__(256, 4) void k_das_adj(DasArgs A) {
  const Geo& g = A.g;
  const int2 w = A.work[blockIdx.x];
  const int tile = w.x, jb = w.y;
  if (tile < 0) return;  // padding item of a shorter XCD queue
  const int4 tr = A.tiles[tile];
  const long long P = g.P;
  const long long p = (long long)tile * TILE + threadIdx.x;
  const int N = g.n_elem, ns = g.ns;
  const float fsf = (float)g.fs;
  const float om = (float)(2.0 * 3.14159265358979323846 * g.fd);

  Rx rx[S];
  int rmin = 0, rmax = 0;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    rx[k] = load_rx(A.tab, P, p, jb * S + k, tr.x, tr.y);
    rmin = min(rmin, rx[k].ui);
    rmax = max(rmax, rx[k].ui);
  }
  float grx[S];
#pragma unroll
  for (int k = 0; k < S; ++k) grx[k] = 0.f;
  const WaveRange wr = wave_range(A.prange, p, tr, jb, S);
  const float gi = A.gscal ? (float)A.gscal[5] : 0.f;
  // DET: this item's slab (workgroup-uniform base), slot (t - tr.x) * TILE + lane point
  float* __restrict__ slab =
      DET ? A.gtp + A.tbase[tile] + (long long)(jb - tr.z) * (tr.y - tr.x + 1) * TILE : nullptr;
  const int me = (int)threadIdx.x - tr.x * TILE;
  const bool busy = wr.rx_active && wr.lo <= wr.hi;
  // transmit elements the wavefront does not visit below hold zero sums
  if (DET)
    for (int t = tr.x; t <= tr.y; ++t)
      if (!busy || t < wr.lo || t > wr.hi) slab[t * TILE + me] = 0.f;
  if (busy) {
    for (int ib = max(tr.z, wr.lo / S); ib <= min(tr.w, wr.hi / S); ++ib) {
      const int t0 = max(ib * S, wr.lo), t1 = min(ib * S + S - 1, wr.hi);
      float2 G = A.gblk[((long long)ib * g.nblk + jb) * P + p];
      if (A.gscal) {  // final scale of the block gradient, as k_gscale forms it
        const float2 sb = A.gsb[p];
        G.x = fmaf(G.x, gi, sb.x);
        G.y = fmaf(G.y, gi, sb.y);
      }
      TabEntry et = A.tab[(long long)t0 * P + p];
      for (int t = t0; t <= t1; ++t) {
        const TabEntry en = A.tab[(long long)min(t + 1, t1) * P + p];
        const bool inside = interior(et, rmin, rmax, ns);
        if (inside || !wave_silent<S>(et, rx, ns)) {
          // Q = conj(G) * E_t
          const float qx = G.x * et.er + G.y * et.ei;
          const float qy = G.x * et.ei - G.y * et.er;
          const float2* __restrict__ base = A.iq + ((long long)t * N + (long long)jb * S) * ns;
          float gtx = 0.f;
          if (inside) das_adj_t<S, false>(base, ns, et, rx, qx, qy, fsf, om, grx, gtx);
          else das_adj_t<S, true>(base, ns, et, rx, qx, qy, fsf, om, grx, gtx);
          if (DET) slab[t * TILE + me] = gtx;
          else if (gtx != 0.f) atomicAdd(A.gT2 + (long long)t * P + p, gtx);
        } else if (DET) {
          slab[t * TILE + me] = 0.f;
        }
        et = en;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const int r = jb * S + k;
    if (r >= tr.x && r <= tr.y) A.gT[(long long)r * P + p] = grx[k];
  }
}

// Receive-channel images X_r(p) = h_r E_r sum_t h_t E_t Psi_{t,r}(u_t + u_r): Eq. 5
// with the transmit aperture the whole array and the receive aperture one element
// (the focused per-channel signals of the coherence metrics).  Same work split
// as k_das_fwd; each lane keeps one accumulator per receive element of its block
// and applies the receive phasor once at the end.
template <int S>
__global__ __launch_bounds__(256) void k_das_rx(DasArgs A, float2* __restrict__ X) {
  const Geo& g = A.g;
  const int2 w = A.work[blockIdx.x];
  const int tile = w.x, jb = w.y;
  if (tile < 0) return;  // padding item of a shorter XCD queue
  const int4 tr = A.tiles[tile];
  const long long P = g.P;
  const long long p = (long long)tile * TILE + threadIdx.x;
  const int N = g.n_elem, ns = g.ns;

  Rx rx[S];
  int rmin = 0, rmax = 0;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    rx[k] = load_rx(A.tab, P, p, jb * S + k, tr.x, tr.y);
    rmin = min(rmin, rx[k].ui);
    rmax = max(rmax, rx[k].ui);
  }
  const WaveRange wr = wave_range(A.prange, p, tr, jb, S);
  const int tlo = wr.rx_active ? wr.lo : tr.y + 1, thi = wr.rx_active ? wr.hi : tr.x - 1;
  float2 acc[S];
#pragma unroll
  for (int k = 0; k < S; ++k) acc[k] = make_float2(0.f, 0.f);
  const RxSpan sp = rx_span<S>(rx);
  for (int t = tlo; t <= thi; ++t) {
    const TabEntry et = A.tab[(long long)t * P + p];
    const bool check = !interior(et, rmin, rmax, ns);
    if (check && wave_silent(et, sp, ns)) continue;
    const float2* __restrict__ base = A.iq + ((long long)t * N + (long long)jb * S) * ns;
    float2 a0[S], a1[S];
    float fr[S];
    bool ok[S];
    if (check) gather<S, true>(base, ns, et, rx, a0, a1, fr, ok);
    else gather<S, false>(base, ns, et, rx, a0, a1, fr, ok);
#pragma unroll
    for (int k = 0; k < S; ++k) {
      float vx = fmaf(fr[k], a1[k].x - a0[k].x, a0[k].x);
      float vy = fmaf(fr[k], a1[k].y - a0[k].y, a0[k].y);
      if (check) {
        vx = ok[k] ? vx : 0.f;
        vy = ok[k] ? vy : 0.f;
      }
      acc[k].x = fmaf(vx, et.er, fmaf(-vy, et.ei, acc[k].x));
      acc[k].y = fmaf(vx, et.ei, fmaf(vy, et.er, acc[k].y));
    }
  }
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const float2 e = rx[k].e;
    X[(long long)(jb * S + k) * P + p] =
        make_float2(acc[k].x * e.x - acc[k].y * e.y, acc[k].x * e.y + acc[k].y * e.x);
  }
}

__global__ __launch_bounds__(256) void k_fill_zero2(float2* __restrict__ x, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    x[i] = make_float2(0.f, 0.f);
}

// Internal -> caller point order of the channel images, one row per element.
__global__ __launch_bounds__(256) void k_export_rx(long long P, long long Pc,
                                                   const int* __restrict__ c2i,
                                                   const float2* __restrict__ X,
                                                   float2* __restrict__ out) {
  const long long pc = (long long)blockIdx.x * 256 + threadIdx.x;
  if (pc >= Pc) return;
  const long long r = blockIdx.y;
  out[r * Pc + pc] = X[r * P + c2i[pc]];
}

// Lag-one coherence of pixel q over its M <= 9 patch points: the mean over
// adjacent receive elements (r, r+1) with energy of
// Re(sum_m X_r conj X_{r+1}) / sqrt(E_r E_{r+1}), E_r = sum_m |X_r|^2; 0 if none.
constexpr float LOC_MIN_ENERGY = 1e-30f;
__global__ __launch_bounds__(256) void k_loc(int N, long long P, int M, int n_pix,
                                             const int* __restrict__ c2i,
                                             const float2* __restrict__ X,
                                             float* __restrict__ loc) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n_pix) return;
  long long pi[9];
  float2 xp[9];
  float ep = 0.f;
#pragma unroll
  for (int m = 0; m < 9; ++m) {
    pi[m] = m < M ? (long long)c2i[(long long)q * M + m] : 0;
    xp[m] = m < M ? X[pi[m]] : make_float2(0.f, 0.f);
    ep = fmaf(xp[m].x, xp[m].x, fmaf(xp[m].y, xp[m].y, ep));
  }
  float sum = 0.f;
  int n = 0;
  for (int r = 1; r < N; ++r) {
    float ec = 0.f, cr = 0.f;
#pragma unroll
    for (int m = 0; m < 9; ++m) {
      const float2 xc = m < M ? X[(long long)r * P + pi[m]] : make_float2(0.f, 0.f);
      ec = fmaf(xc.x, xc.x, fmaf(xc.y, xc.y, ec));
      cr = fmaf(xp[m].x, xc.x, fmaf(xp[m].y, xc.y, cr));
      xp[m] = xc;
    }
    if (ep > LOC_MIN_ENERGY && ec > LOC_MIN_ENERGY) {
      sum += cr / (sqrtf(ep) * sqrtf(ec));
      ++n;
    }
    ep = ec;
  }
  loc[q] = n > 0 ? sum / (float)n : 0.f;
}

// Zero the transmit-role sums over the active elements of every tile.
__global__ __launch_bounds__(256) void k_zero_tx(Geo g, const int4* __restrict__ tiles,
                                                 float* __restrict__ gT2) {
  const int tile = blockIdx.x;
  const int4 tr = tiles[tile];
  const long long p = (long long)tile * TILE + threadIdx.x;
  for (int a = tr.x; a <= tr.y; ++a) gT2[(long long)a * g.P + p] = 0.f;
}

template <int S>
hipError_t das_fwd_s(af_ctx* c, const DasArgs& A) {
  hipLaunchKernelGGL(k_das_fwd<S>, dim3(c->v.n_das_work), dim3(256), 0, c->stream, A);
  return hipGetLastError();
}

template <int S>
hipError_t das_adj_s(af_ctx* c, const DasArgs& A) {
  if (c->det) {
    hipLaunchKernelGGL((k_das_adj<S, true>), dim3(c->v.n_das_work), dim3(256), 0, c->stream, A);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_zero_tx, dim3(c->v.n_tiles), dim3(256), 0, c->stream, A.g, A.tiles, A.gT2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_das_adj<S, false>), dim3(c->v.n_das_work), dim3(256), 0, c->stream, A);
  return hipGetLastError();
}

DasArgs das_args(af_ctx* c, const float2* iq) {
  DasArgs A{};
  A.g = c->geo();
  A.tab = c->d_tab.as<TabEntry>();
  A.iq = iq;
  A.tiles = c->v.tiles;
  A.prange = c->v.prange;
  A.work = c->v.daswork;
  A.order = c->v.order;
  return A;
}

}  // namespace

hipError_t launch_das_fwd(af_ctx* c, const float2* iq, float2* bblk) {
  if (c->v.n_das_work == 0) return hipSuccess;
  DasArgs A = das_args(c, iq);
  A.bblk = bblk;
  switch (c->S) {
    case 1: return das_fwd_s<1>(c, A);
    case 2: return das_fwd_s<2>(c, A);
    case 4: return das_fwd_s<4>(c, A);
    case 8: return das_fwd_s<8>(c, A);
    case 16: return das_fwd_s<16>(c, A);
    default: return hipErrorInvalidValue;
  }
}

template <int S>
hipError_t das_rx_s(af_ctx* c, const DasArgs& A, float2* X) {
  hipLaunchKernelGGL(k_das_rx<S>, dim3(c->v.n_das_work), dim3(256), 0, c->stream, A, X);
  return hipGetLastError();
}

hipError_t launch_channel_images(af_ctx* c, const float2* iq, float2* X) {
  const long long n = (long long)c->N * c->P_int;
  const unsigned nblk = (unsigned)std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_fill_zero2, dim3(std::max(nblk, 1u)), dim3(256), 0, c->stream, X, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || c->v.n_das_work == 0) return e;
  DasArgs A = das_args(c, iq);
  switch (c->S) {
    case 1: return das_rx_s<1>(c, A, X);
    case 2: return das_rx_s<2>(c, A, X);
    case 4: return das_rx_s<4>(c, A, X);
    case 8: return das_rx_s<8>(c, A, X);
    case 16: return das_rx_s<16>(c, A, X);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_export_rx(af_ctx* c, const float2* X, float2* out) {
  const long long Pc = c->P;
  hipLaunchKernelGGL(k_export_rx, dim3((unsigned)((Pc + 255) / 256), (unsigned)c->N), dim3(256), 0,
                     c->stream, (long long)c->P_int, Pc, c->d_c2i.as<int>(), X, out);
  return hipGetLastError();
}

hipError_t launch_loc(af_ctx* c, const float2* X, float* loc) {
  hipLaunchKernelGGL(k_loc, dim3((unsigned)((c->n_pix + 255) / 256)), dim3(256), 0, c->stream, c->N,
                     (long long)c->P_int, c->M, c->n_pix, c->d_c2i.as<int>(), X, loc);
  return hipGetLastError();
}

hipError_t launch_das_adj(af_ctx* c, const float2* iq, const float2* gblk, bool scaled) {
  if (c->v.n_das_work == 0) return hipSuccess;
  DasArgs A = das_args(c, iq);
  A.gblk = gblk;
  A.gscal = scaled ? nullptr : c->d_scal.as<double>();
  A.gsb = c->v.gsb;
  A.gT = c->d_gT.as<float>();
  A.gT2 = c->d_gT.as<float>() + (size_t)c->N * c->v.P;
  A.gtp = c->d_gtp.as<float>();
  A.tbase = c->v.tbase;
  switch (c->S) {
    case 1: return das_adj_s<1>(c, A);
    case 2: return das_adj_s<2>(c, A);
    case 4: return das_adj_s<4>(c, A);
    case 8: return das_adj_s<8>(c, A);
    case 16: return das_adj_s<16>(c, A);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace af
