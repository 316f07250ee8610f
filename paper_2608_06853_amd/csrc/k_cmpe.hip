// Common-midpoint phase error on subaperture images built from block pairs, its
// gradient with respect to the block images, speckle brightness, coherence
// factor and the per-pixel integrated CMPE map (Objective Function subsection;
// Model Implementation: 3x3 patches at lambda/2).
//
// Reading of the CMPE (the exact definition is in the cited Simson et al.
// paper): subaperture i spans blocks {i, i+1}; the common-midpoint neighbour
// pair (i, j) compares X = B_{i,j+1} and Y = B_{i+1,j} over a patch through
// C = sum X conj(Y); it is valid when both energies exceed 1e-30 and
// rho = |C| / sqrt(sum|X|^2 sum|Y|^2) >= rho_thresh; its error is |arg C|.
//
// Four wavefronts own one sub-tile of 64 points (whole patches plus padding) and
// stage its subaperture images in LDS.  Partial sums go to a per-sub-tile slot
// and are reduced in fixed order afterwards (deterministic).  A tile whose span
// of active blocks is too wide for LDS (deep points of a linear array see every
// block) runs the same code in a second launch with the staging area in device
// memory.
#include "af_internal.h"

namespace af {
namespace {

// Smallest energy sum|X|^2 of a valid pair: below it |C|^2 leaves the FP32 range.
constexpr float kMinEnergy = 1e-30f;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

constexpr int CMPE_WAVES = 4;
// Row stride (float2) of a subaperture image in LDS: one more than the sub-tile, so
// the rows that neighbouring pair entries read start two banks apart.
constexpr int SS = SUB + 1;

// Dynamic LDS (float2) of a sub-tile whose tile spans blocks bLO..bHI: the (npr +
// 1)^2 subaperture images at row stride SS, then pps x npr^2 pair entries of one
// float2 and two floats (the layout below).
__device__ __host__ inline long long cmpe_lds_need(int bLO, int bHI, int nsub, int pps) {
  const int pLo = bLO - 1 > 0 ? bLO - 1 : 0;
  const int pHi = nsub - 2 < bHI - 1 ? nsub - 2 : bHI - 1;
  const long long npr = pHi - pLo + 1 > 0 ? pHi - pLo + 1 : 0;
  const long long nS = npr > 0 ? npr + 1 : 0;
  return nS * nS * SS + 2LL * pps * npr * npr;
}

// One workgroup of 4 wavefronts per 64-point sub-tile.  Phase 1 forms, for this
// sub-tile, the full image and block energy per point and every subaperture
// image S(i, j) = sum of its 2 x 2 block images that a pair of the sub-tile can
// use, in LDS.  Phase 2 evaluates the (pixel, pair) entries; phase 3 writes the
// gradient of every active block image as the sum of dL/dS over the four
// subapertures that contain it.  The block images are read only in phase 1, so
// the gradient may overwrite them in place.  WIDE: only the tiles of the
// device-memory path, whose staging area is their slice of A.wscr.
template <bool WIDE>
__global__ __launch_bounds__(256) void k_cmpe(CmpeArgs A) {
  extern __shared__ float2 sm[];
  __shared__ float pimg[CMPE_WAVES][3][SUB];
  __shared__ double red[CMPE_WAVES][3];
  const Geo& g = A.g;
  const int tid = threadIdx.x, lane = tid & (SUB - 1), wv = tid / SUB;
  const long long st = blockIdx.x;
  const long long p0 = st * SUB;
  const long long tile = p0 / TILE;
  const int w = (int)((p0 % TILE) / SUB);
  const int4 tr = A.tiles[tile];
  const int wix = A.wide[tile];
  if ((wix >= 0) != WIDE) return;  // the other launch owns this sub-tile
  const int M = g.patch2, pps = g.pps;
  if (!WIDE) {  // the LDS path: the launch whose LDS class holds this tile's need
    const long long need = tr.x <= tr.y ? cmpe_lds_need(tr.z, tr.w, g.nsub, pps) : 0;
    if (need <= A.need_lo || need > A.need_hi) return;
  }
  const long long P = g.P;
  const long long slot0 = tile * (4 * pps) + (long long)w * pps;

  if (tr.x > tr.y) {  // (a tile without work is never wide)
    if (tid < SUB) {
      A.gsb[p0 + tid] = make_float2(0.f, 0.f);
      if (A.img) A.img[p0 + tid] = make_float2(0.f, 0.f);
      if (tid < pps) {
        if (A.map_cmpe) A.map_cmpe[slot0 + tid] = 0.f;
        if (A.map_cf) A.map_cf[slot0 + tid] = 0.f;
        if (A.map_cmcc) A.map_cmcc[slot0 + tid] = 0.f;
      }
    }
    if (tid == 0) {
      A.part[4 * st + 0] = 0.0;
      A.part[4 * st + 1] = 0.0;
      A.part[4 * st + 2] = 0.0;
      A.part[4 * st + 3] = 0.0;
    }
    return;
  }
  const int bLO = tr.z, bHI = tr.w, nbA = bHI - bLO + 1, nbb = nbA * nbA;
  // pairs (i, j) in [pLo, pHi]^2 use subapertures with indices in [pLo, pHi + 1]
  const int pLo = max(0, bLO - 1);
  const int pHi = min(g.nsub - 2, bHI - 1);
  const int npr = max(0, pHi - pLo + 1);
  const int np2 = npr * npr;
  const int nS = npr > 0 ? npr + 1 : 0;
  float2* Ss = WIDE ? A.wscr + (long long)(wix * 4 + w) * A.wstride : sm;  // [nS * nS][SS]
  float2* gC = Ss + (size_t)nS * nS * SS;            // [pps][np2]
  float* er = reinterpret_cast<float*>(gC + (size_t)pps * np2);
  float* rh = er + (size_t)pps * np2;                // rho of each entry, -1 if no energy

  auto bget = [&](int a, int b) -> float2 {
    if (a < bLO || a > bHI || b < bLO || b > bHI) return make_float2(0.f, 0.f);
    return A.bblk[((long long)a * g.nblk + b) * P + p0 + lane];
  };

  // phase 1: per-point image and energy (a quarter of the blocks per wavefront),
  // subaperture images
  {
    float bx = 0.f, by = 0.f, e2 = 0.f;
    for (int b = wv; b < nbb; b += CMPE_WAVES) {
      const float2 v = A.bblk[((long long)(bLO + b / nbA) * g.nblk + (bLO + b % nbA)) * P + p0 + lane];
      bx += v.x;
      by += v.y;
      e2 += v.x * v.x + v.y * v.y;
    }
    pimg[wv][0][lane] = bx;
    pimg[wv][1][lane] = by;
    pimg[wv][2][lane] = e2;
  }
  for (int idx = wv; idx < nS * nS; idx += CMPE_WAVES) {
    const int si = pLo + idx / nS, sj = pLo + idx % nS;
    const float2 a = bget(si, sj), b = bget(si + 1, sj), c = bget(si, sj + 1), d = bget(si + 1, sj + 1);
    Ss[(size_t)idx * SS + lane] = make_float2(a.x + b.x + c.x + d.x, a.y + b.y + c.y + d.y);
  }
  __syncthreads();

  // phase 2: (pixel, pair) entries
  double e_acc = 0.0, nv = 0.0;
  for (int item = tid; item < pps * np2; item += CMPE_WAVES * SUB) {
    const int q = item / np2, pr = item - q * np2;
    const int i = pLo + pr / npr, j = pLo + pr % npr;
    const float2* Xs = Ss + (size_t)((i - pLo) * nS + (j + 1 - pLo)) * SS + q * M;
    const float2* Ys = Ss + (size_t)((i + 1 - pLo) * nS + (j - pLo)) * SS + q * M;
    float cx = 0.f, cy = 0.f, ex = 0.f, ey = 0.f;
    for (int m = 0; m < M; ++m) {
      const float2 X = Xs[m], Y = Ys[m];
      cx += X.x * Y.x + X.y * Y.y;
      cy += X.y * Y.x - X.x * Y.y;
      ex += X.x * X.x + X.y * X.y;
      ey += Y.x * Y.x + Y.y * Y.y;
    }
    const float mag = sqrtf(cx * cx + cy * cy);
    bool valid = ex > kMinEnergy && ey > kMinEnergy;
    const float rho = valid ? mag / (sqrtf(ex) * sqrtf(ey)) : -1.f;
    rh[item] = rho;
    if (valid) valid = rho >= A.rho_thresh;
    const float ang = atan2f(cy, cx);
    float2 gc = make_float2(0.f, 0.f);
    if (valid) {
      // d|arg C|/dC = sign(arg C) j C / |C|^2, formed as (j C/|C|) (sign/|C|) so that
      // no intermediate leaves the FP32 range
      if (ang != 0.f && mag > kMinEnergy) {
        const float im = 1.f / mag;
        const float sg = ang > 0.f ? im : -im;
        gc = make_float2(-cy * im * sg, cx * im * sg);
      }
      e_acc += fabsf(ang);
      nv += 1.0;
    }
    gC[item] = gc;
    er[item] = valid ? fabsf(ang) : -1.f;
  }
  __syncthreads();

  if (tid < pps && A.map_cmpe) {
    float s = 0.f;
    int n = 0;
    for (int k = 0; k < np2; ++k) {
      const float e = er[tid * np2 + k];
      if (e >= 0.f) {
        s += e;
        ++n;
      }
    }
    A.map_cmpe[slot0 + tid] = n > 0 ? s / (float)n : 0.f;
  }
  if (tid < pps && A.map_cmcc) {  // common-midpoint correlation coefficient
    float s = 0.f;
    int n = 0;
    for (int k = 0; k < np2; ++k) {
      const float r = rh[tid * np2 + k];
      if (r >= 0.f) {
        s += r;
        ++n;
      }
    }
    A.map_cmcc[slot0 + tid] = n > 0 ? s / (float)n : 0.f;
  }

  // phase 3: dL/dB(i0, j0) = sum over the subapertures (i, j), i in {i0-1, i0},
  // j in {j0-1, j0}, of dL/dS(i, j), where S(i, j) is X of pair (i, j-1) and Y of
  // pair (i-1, j)
  if (A.write_g) {
    for (int b = wv; b < nbb; b += CMPE_WAVES) {
      const int i0 = bLO + b / nbA, j0 = bLO + b % nbA;
      float2 G = make_float2(0.f, 0.f);
      if (lane < pps * M && npr > 0) {
        const int q = lane / M;
        const float2* gq = gC + q * np2;
        for (int di = -1; di <= 0; ++di)
          for (int dj = -1; dj <= 0; ++dj) {
            const int i = i0 + di, j = j0 + dj;
            if (i < 0 || j < 0 || i > g.nsub - 1 || j > g.nsub - 1) continue;
            if (i >= pLo && i <= pHi && j - 1 >= pLo && j - 1 <= pHi) {
              const float2 c = gq[(i - pLo) * npr + (j - 1 - pLo)];
              const float2 y = Ss[(size_t)((i + 1 - pLo) * nS + (j - 1 - pLo)) * SS + lane];
              G.x += c.x * y.x - c.y * y.y;
              G.y += c.x * y.y + c.y * y.x;
            }
            if (i - 1 >= pLo && i - 1 <= pHi && j >= pLo && j <= pHi) {
              const float2 c = gq[(i - 1 - pLo) * npr + (j - pLo)];
              const float2 x = Ss[(size_t)((i - 1 - pLo) * nS + (j + 1 - pLo)) * SS + lane];
              G.x += c.x * x.x + c.y * x.y;
              G.y += c.x * x.y - c.y * x.x;
            }
          }
      }
      A.gout[((long long)i0 * g.nblk + j0) * P + p0 + lane] = G;
    }
  }

  // full image, speckle brightness and coherence factor at each point
  double sbp = 0.0;
  if (wv == 0) {
    float bx = 0.f, by = 0.f, e2 = 0.f;
    for (int k = 0; k < CMPE_WAVES; ++k) {
      bx += pimg[k][0][lane];
      by += pimg[k][1][lane];
      e2 += pimg[k][2][lane];
    }
    if (A.img) A.img[p0 + lane] = make_float2(bx, by);
    const bool centre = lane < pps * M && (lane % M) == M / 2;
    if (centre) {
      const float b2 = bx * bx + by * by;
      sbp = (double)b2;
      if (A.map_cf)
        A.map_cf[slot0 + lane / M] = e2 > 0.f ? b2 / ((float)g.nblk * (float)g.nblk * e2) : 0.f;
      A.gsb[p0 + lane] = make_float2(A.sb_scale * bx, A.sb_scale * by);
    } else {
      A.gsb[p0 + lane] = make_float2(0.f, 0.f);
    }
  }
  e_acc = wave_sum(e_acc);
  nv = wave_sum(nv);
  sbp = wave_sum(sbp);
  if (lane == 0) {
    red[wv][0] = e_acc;
    red[wv][1] = nv;
    red[wv][2] = sbp;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k = 0; k < CMPE_WAVES; ++k) {
      a += red[k][0];
      b += red[k][1];
      c += red[k][2];
    }
    A.part[4 * st + 0] = a;
    A.part[4 * st + 1] = b;
    A.part[4 * st + 2] = c;
    A.part[4 * st + 3] = 0.0;
  }
}

// Internal -> caller order: travel times of the caller points whose internal
// point lies in the view [p0, p0 + g.P) (the table holds that view).
__global__ __launch_bounds__(256) void k_export_T(Geo g, const TabEntry* __restrict__ tab,
                                                  const int* __restrict__ c2i,
                                                  const int2* __restrict__ prange, long long Pc,
                                                  long long p0, float* __restrict__ out) {
  const long long pc = (long long)blockIdx.x * 256 + threadIdx.x;
  const int a = blockIdx.y;
  if (pc >= Pc) return;
  const long long p = c2i[pc];
  if (p < p0 || p >= p0 + g.P) return;
  const int2 pr = prange[p];
  float v = __int_as_float(0x7fc00000);
  if (a >= pr.x && a <= pr.y) {
    const TabEntry e = tab[(long long)a * g.P + (p - p0)];
    const double u = (double)e.ui + (double)e.uf;
    v = (float)(u / g.fs - 0.5 * g.t_ttp + 0.5 * g.t0);
  }
  out[(long long)a * Pc + pc] = v;
}

// Internal -> caller order: block images, full image and per-pixel maps of the
// caller points whose internal point lies in the view [p0, p0 + g.P) (the block
// images hold that view; tiles and maps are the whole arrays).
__global__ __launch_bounds__(256) void k_export_img(Geo g, const float2* __restrict__ bblk,
                                                    const int4* __restrict__ tiles,
                                                    const int* __restrict__ c2i, long long Pc,
                                                    long long p0,
                                                    int n_pix, const float* __restrict__ mc,
                                                    const float* __restrict__ mcf,
                                                    const float* __restrict__ mcc,
                                                    float2* __restrict__ blk_out,
                                                    float2* __restrict__ img_out,
                                                    float* __restrict__ maps_out) {
  const long long pc = (long long)blockIdx.x * 256 + threadIdx.x;
  if (pc >= Pc) return;
  const long long p = c2i[pc];
  if (p < p0 || p >= p0 + g.P) return;
  const int4 tr = tiles[p / TILE];
  float2 acc = make_float2(0.f, 0.f);
  for (int i = 0; i < g.nblk; ++i)
    for (int j = 0; j < g.nblk; ++j) {
      float2 v = make_float2(0.f, 0.f);
      if (tr.x <= tr.y && i >= tr.z && i <= tr.w && j >= tr.z && j <= tr.w)
        v = bblk[((long long)i * g.nblk + j) * g.P + (p - p0)];
      acc.x += v.x;
      acc.y += v.y;
      if (blk_out) blk_out[((long long)i * g.nblk + j) * Pc + pc] = v;
    }
  if (img_out) img_out[pc] = acc;
  if (maps_out && (pc % g.patch2) == g.patch2 / 2) {
    const long long l = p % TILE;
    const long long slot = (p / TILE) * 4 * g.pps + (l / SUB) * g.pps + (l % SUB) / g.patch2;
    const long long q = pc / g.patch2;
    maps_out[q] = mc[slot];
    maps_out[n_pix + q] = mcf[slot];
    maps_out[2 * (long long)n_pix + q] = mcc[slot];
  }
}

}  // namespace

long long cmpe_wide_stride(int nba, int pps) {
  // the dynamic LDS layout of k_cmpe for a span of nba blocks, in float2: the
  // subaperture images, then pps * nba^2 pair entries of one float2 and two floats
  return (long long)(nba + 1) * (nba + 1) * SS + 2LL * pps * nba * nba;
}

long long cmpe_need(int bLO, int bHI, int nsub, int pps) { return cmpe_lds_need(bLO, bHI, nsub, pps); }

bool cmpe_fits_lds(int bLO, int bHI, int nsub, int pps) {
  const size_t budget = 160 * 1024 - sizeof(float) * CMPE_WAVES * 3 * SUB -
                        sizeof(double) * CMPE_WAVES * 3 - 256;
  return sizeof(float2) * (size_t)cmpe_lds_need(bLO, bHI, nsub, pps) <= budget;
}

hipError_t launch_cmpe(af_ctx* c, const float2* bblk, float2* gout, int write_g, float rho,
                       float sb_scale, float* map_cmpe, float* map_cf, float* map_cmcc,
                       float2* img) {
  CmpeArgs A{};
  A.g = c->geo();
  A.tiles = c->v.tiles;
  A.bblk = bblk;
  A.gout = gout;
  A.gsb = c->v.gsb;
  A.part = c->v.part;
  A.map_cmpe = map_cmpe;
  A.map_cf = map_cf;
  A.map_cmcc = map_cmcc;
  A.img = img;
  A.rho_thresh = rho;
  A.sb_scale = sb_scale;
  A.write_g = write_g;
  A.wide = c->v.wide;
  A.wscr = c->d_cmpe_wide.as<float2>();
  A.wstride = c->wstride;
  const long long most = std::max(c->need_lds, 1LL);  // the largest need on the LDS path
  const dim3 grid((unsigned)(c->v.P / SUB)), block(CMPE_WAVES * SUB);
  // Tiles of a narrow span run with an allocation that lets six workgroups share a
  // CU; the wider ones with the widest span's (one launch when that is small).
  const long long narrow =
      ((long long)(160 * 1024 / 6) - (long long)(sizeof(float) * CMPE_WAVES * 3 * SUB +
                                                 sizeof(double) * CMPE_WAVES * 3)) /
      (long long)sizeof(float2);
  const long long cut = most <= narrow ? most : narrow;
  A.need_lo = -1;
  A.need_hi = cut;
  hipLaunchKernelGGL(k_cmpe<false>, grid, block, sizeof(float2) * (size_t)cut, c->stream, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (most > cut) {
    A.need_lo = cut;
    A.need_hi = most;
    hipLaunchKernelGGL(k_cmpe<false>, grid, block, sizeof(float2) * (size_t)most, c->stream, A);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (c->v.n_wide == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cmpe<true>, grid, block, 0, c->stream, A);
  return hipGetLastError();
}

hipError_t launch_export_T(af_ctx* c, float* out) {
  const long long Pc = c->P;
  dim3 grid((unsigned)((Pc + 255) / 256), (unsigned)c->N);
  hipLaunchKernelGGL(k_export_T, grid, dim3(256), 0, c->stream, c->geo(), c->d_tab.as<TabEntry>(),
                     c->d_c2i.as<int>(), c->d_prange.as<int2>(), Pc, c->v.p0, out);
  return hipGetLastError();
}

hipError_t launch_export_images(af_ctx* c, const float2* bblk, float2* blk_out, float2* img_out,
                                float* maps_out) {
  const long long Pc = c->P;
  hipLaunchKernelGGL(k_export_img, dim3((unsigned)((Pc + 255) / 256)), dim3(256), 0, c->stream,
                     c->geo(), bblk, c->d_tiles.as<int4>(), c->d_c2i.as<int>(), Pc, c->v.p0,
                     c->n_pix,
                     c->d_maps.as<float>(), c->d_maps.as<float>() + c->n_tiles * c->ppt,
                     c->d_maps.as<float>() + 2 * (size_t)c->n_tiles * c->ppt, blk_out, img_out,
                     maps_out);
  return hipGetLastError();
}

}  // namespace af
