// Host side of the C ABI: context, geometry set-up (element orientation, active
// element ranges, spatial tiling of the evaluation points, work lists), buffer
// management and the sequence of kernels behind each entry point.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <thread>

#include "af_internal.h"

using af::DBuf;
using af::TILE;
using af::SUB;

namespace {

const char* kNoCtx = "af: null context";
// why the last af_create of this thread failed (af_last_error(NULL) returns it)
thread_local std::string g_create_err;

af_status fail(af_ctx* c, af_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

af_status hip_fail(af_ctx* c, hipError_t e, const char* where) {
  return fail(c, AF_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define AF_HIP(call, where)                                   \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return hip_fail(c, e_, where);      \
  } while (0)

// Launch `call` (a launch wrapper) and, when profiling, bracket it with events.
#define AF_KERNEL(kid, call, where)                                            \
  do {                                                                         \
    hipEvent_t a_ = nullptr, b_ = nullptr;                                     \
    if (c->prof_on && (a_ = c->ev_get())) (void)hipEventRecord(a_, c->stream); \
    AF_HIP(call, where);                                                       \
    if (a_ && (b_ = c->ev_get())) {                                            \
      (void)hipEventRecord(b_, c->stream);                                     \
      c->ev_pending.push_back({(kid), {a_, b_}});                              \
    } else if (a_) {                                                           \
      c->ev_pool.push_back(a_);                                                \
    }                                                                          \
  } while (0)

#define AF_ALLOC(buf, bytes, what)                                                    \
  do {                                                                                \
    if ((buf).ensure(bytes) != hipSuccess)                                            \
      return fail(c, AF_ERR_OOM, std::string("af: cannot allocate ") + (what));       \
  } while (0)

// Host worker threads for the per-point loops of the geometry set-up.
int host_threads(long long work) {
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  return (int)std::max<long long>(1, std::min<long long>(hw, work / 65536));
}

// Runs fn(t, nthr) on nthr threads (thread 0 is the caller).  Workers keep
// their running results in locals and write them once (no shared cache lines
// are updated inside the loops).
template <class F>
void parallel(int nthr, F&& fn) {
  std::vector<std::thread> pool;
  for (int t = 1; t < nthr; ++t) pool.emplace_back(fn, t, nthr);
  fn(0, nthr);
  for (auto& t : pool) t.join();
}

// Orders idx[0..n) so that consecutive runs of `unit` items (and of `sub` items
// inside them) are spatially compact: recursive median split along the longer
// extent of (u, v), with the left part always a whole number of units.  The two
// halves of the top `par_depth` levels are split on separate threads (the
// result does not depend on it).
void kd_partition(int* idx, int n, int unit, int sub, const std::vector<double>& u,
                  const std::vector<double>& v, int par_depth = 0) {
  if (n <= sub) return;
  const int q = n > unit ? unit : sub;
  const int n_left = q * ((n + 2 * q - 1) / (2 * q));
  if (n_left >= n) return;
  double ulo = 1e300, uhi = -1e300, vlo = 1e300, vhi = -1e300;
  for (int k = 0; k < n; ++k) {
    ulo = std::min(ulo, u[idx[k]]);
    uhi = std::max(uhi, u[idx[k]]);
    vlo = std::min(vlo, v[idx[k]]);
    vhi = std::max(vhi, v[idx[k]]);
  }
  const std::vector<double>& key = (uhi - ulo) >= (vhi - vlo) ? u : v;
  std::nth_element(idx, idx + n_left, idx + n, [&](int a, int b) {
    return key[a] < key[b] || (key[a] == key[b] && a < b);
  });
  if (par_depth > 0 && n > 20000) {
    std::thread left(kd_partition, idx, n_left, unit, sub, std::cref(u), std::cref(v),
                     par_depth - 1);
    kd_partition(idx + n_left, n - n_left, unit, sub, u, v, par_depth - 1);
    left.join();
  } else {
    kd_partition(idx, n_left, unit, sub, u, v, 0);
    kd_partition(idx + n_left, n - n_left, unit, sub, u, v, 0);
  }
}

// Every node of a slowness grid on the device must be finite and positive: reads
// the n values back (the stream is synchronised) and checks them on the host.
af_status check_slowness(af_ctx* c, const float* s_dev, size_t n, const char* who) {
  std::vector<float> h(n);
  AF_HIP(hipMemcpyAsync(h.data(), s_dev, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream), who);
  AF_HIP(hipStreamSynchronize(c->stream), who);
  for (size_t i = 0; i < n; ++i)
    if (!(h[i] > 0.f) || !std::isfinite(h[i]))
      return fail(c, AF_ERR_NUMERIC,
                  std::string(who) + ": slowness node " + std::to_string(i) +
                      " is not finite and positive");
  return AF_OK;
}

template <class T>
af_status upload(af_ctx* c, DBuf& b, const std::vector<T>& v, const char* what) {
  AF_ALLOC(b, sizeof(T) * std::max<size_t>(v.size(), 1), what);
  if (!v.empty())
    AF_HIP(hipMemcpyAsync(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, c->stream), what);
  // host vectors die at return: wait for the copy
  AF_HIP(hipStreamSynchronize(c->stream), what);
  return AF_OK;
}

// Device bytes of the chunk-sized buffers per point: table entry, ray start and
// medium leg, the two dL/dT roles per element, and the block images.
size_t bytes_per_point(const af_ctx* c) {
  return (size_t)c->N * (sizeof(af::TabEntry) + sizeof(float2) + 3 * sizeof(float)) +
         (size_t)c->nb * c->nb * sizeof(float2);
}

// From the active element range of every tile (c->tile_lo, c->tile_hi): the tile
// descriptors (element and block ranges); the chunks of consecutive tiles (one
// chunk unless a memory budget is set); for every chunk, with chunk-local tile
// indices, the table work list (TAB_CHUNK elements per tile), the DAS work list,
// the heaviest-first tile order of the adjoints, the slab offsets of the
// deterministic mode and the CMPE stage's split into LDS and device-memory tiles;
// uploads them and sizes the chunk buffers.
af_status build_work_lists(af_ctx* c) {
  const int n_tiles = c->n_tiles, block = c->S;
  std::vector<int4> tiles(n_tiles);
  c->na_max = 1;
  c->nba_max = 1;
  for (int t = 0; t < n_tiles; ++t) {
    const int LO = c->tile_lo[t], HI = c->tile_hi[t];
    if (LO > HI) {
      tiles[t] = make_int4(1, 0, 1, 0);
      continue;
    }
    const int bLO = LO / block, bHI = HI / block;
    tiles[t] = make_int4(LO, HI, bLO, bHI);
    c->na_max = std::max(c->na_max, HI - LO + 1);
    c->nba_max = std::max(c->nba_max, bHI - bLO + 1);
  }
  // CMPE stage: tiles whose staging does not fit LDS take the device-memory path
  c->wstride = af::cmpe_wide_stride(c->nba_max, c->pps);
  c->need_lds = 1;
  c->n_wide = 0;
  std::vector<char> is_wide(std::max(n_tiles, 1), 0);
  for (int t = 0; t < n_tiles; ++t) {
    const int4 tr = tiles[t];
    if (tr.x > tr.y) continue;
    if (!af::cmpe_fits_lds(tr.z, tr.w, c->nsub, c->pps)) {
      is_wide[t] = 1;
      ++c->n_wide;
    } else {
      c->need_lds = std::max(c->need_lds, af::cmpe_need(tr.z, tr.w, c->nsub, c->pps));
    }
  }
  auto slab_floats = [&](int t) {
    const int4 tr = tiles[t];
    return tr.x > tr.y ? 0LL : (long long)(tr.w - tr.z + 1) * (tr.y - tr.x + 1) * af::TILE;
  };
  // chunks: consecutive tiles while their buffers fit the budget (at least one tile)
  c->chunks.clear();
  {
    const size_t per_tile = af::TILE * bytes_per_point(c);
    const size_t wide_bytes = sizeof(float2) * 4 * (size_t)c->wstride;
    af::Chunk ch;
    size_t used = 0;
    for (int t = 0; t < n_tiles; ++t) {
      const size_t need = per_tile + (is_wide[t] ? wide_bytes : 0) +
                          (c->det ? sizeof(float) * (size_t)slab_floats(t) : 0);
      if (c->mem_budget > 0 && ch.n_tiles > 0 && used + need > c->mem_budget) {
        c->chunks.push_back(ch);
        ch = af::Chunk();
        ch.t0 = t;
        used = 0;
      }
      ++ch.n_tiles;
      used += need;
    }
    c->chunks.push_back(ch);  // (an empty chunk when there are no tiles)
  }
  std::vector<int2> tabwork, daswork;
  std::vector<int> order, wide(std::max(n_tiles, 1), -1);
  std::vector<long long> tbase(std::max(n_tiles, 1), 0);
  c->P_chunk = 0;
  c->wide_max = 0;
  c->gtp_max = 0;
  for (af::Chunk& ch : c->chunks) {
    const int t0 = ch.t0, t1 = ch.t0 + ch.n_tiles;
    c->P_chunk = std::max(c->P_chunk, (long long)ch.n_tiles * af::TILE);
    ch.tab_off = (int)tabwork.size();
    ch.das_off = (int)daswork.size();
    ch.ord_off = (int)order.size();
    std::vector<std::pair<long long, int>> load;
    for (int t = t0; t < t1; ++t) {
      const int4 tr = tiles[t];
      if (tr.x > tr.y) continue;
      for (int a0 = tr.x; a0 <= tr.y; a0 += af::TAB_CHUNK) tabwork.push_back(make_int2(t - t0, a0));
      load.push_back({(long long)(tr.y - tr.x + 1) * (tr.y - tr.x + 1), t - t0});
      if (is_wide[t]) wide[t] = ch.n_wide++;
      tbase[t] = ch.n_gtp;
      ch.n_gtp += slab_floats(t);
    }
    std::stable_sort(load.begin(), load.end(), [](auto& a, auto& b) { return a.first > b.first; });
    for (auto& l : load) order.push_back(l.second);
    // DAS work items (tile, receive block).  Workgroups are dealt to the XCDs
    // round-robin (workgroup b runs on XCD b % 8).  The tiles with work, in k-d
    // (spatial) order, are cut into runs of 16 that are dealt to the XCDs in turn,
    // and all receive blocks of a tile go to the same XCD, one after another: the
    // table entries of a tile, which every one of its items reads, are then
    // fetched into one XCD's L2 once, and the 16 neighbouring tiles of a run reuse
    // their channel-data windows there.  Runs of 16 (rather than one long run per
    // XCD) keep the eight queues close in length when the work per tile varies
    // across the image.  Shorter queues are padded with empty items (tile -1).
    constexpr int NXCD = 8, RUN = 16;
    std::vector<std::vector<int2>> q(NXCD);
    int n_live = 0;
    for (int t = t0; t < t1; ++t) {
      const int4 tr = tiles[t];
      if (tr.x > tr.y) continue;
      const int x = (n_live++ / RUN) % NXCD;
      for (int jb = tr.z; jb <= tr.w; ++jb) q[x].push_back(make_int2(t - t0, jb));
    }
    size_t L = 0;
    for (auto& w : q) L = std::max(L, w.size());
    for (size_t i = 0; i < L; ++i)
      for (int x = 0; x < NXCD; ++x) daswork.push_back(i < q[x].size() ? q[x][i] : make_int2(-1, 0));
    ch.n_tab = (int)tabwork.size() - ch.tab_off;
    ch.n_das = (int)daswork.size() - ch.das_off;
    ch.n_ord = (int)order.size() - ch.ord_off;
    c->wide_max = std::max(c->wide_max, ch.n_wide);
    c->gtp_max = std::max(c->gtp_max, ch.n_gtp);
  }
  af_status st;
  if ((st = upload(c, c->d_tiles, tiles, "tiles")) != AF_OK) return st;
  if ((st = upload(c, c->d_tabwork, tabwork, "work list")) != AF_OK) return st;
  if ((st = upload(c, c->d_daswork, daswork, "work list")) != AF_OK) return st;
  if ((st = upload(c, c->d_order, order, "tile order")) != AF_OK) return st;
  if ((st = upload(c, c->d_wide, wide, "wide tiles")) != AF_OK) return st;
  if ((st = upload(c, c->d_tbase, tbase, "slab offsets")) != AF_OK) return st;
  // the chunk-sized buffers
  const size_t Pc = (size_t)std::max(c->P_chunk, 1LL), N = (size_t)c->N;
  AF_ALLOC(c->d_tab, sizeof(af::TabEntry) * N * Pc, "travel-time table");
  AF_ALLOC(c->d_ray_uv, sizeof(float2) * N * Pc, "ray starts");
  AF_ALLOC(c->d_ray_l2, sizeof(float) * N * Pc, "ray medium legs");
  AF_ALLOC(c->d_bblk, sizeof(float2) * (size_t)c->nb * c->nb * Pc, "block images");
  AF_ALLOC(c->d_gT, sizeof(float) * 2 * N * Pc, "time gradient");
  if (c->wide_max > 0)
    AF_ALLOC(c->d_cmpe_wide, sizeof(float2) * 4 * (size_t)c->wide_max * c->wstride,
             "CMPE staging of wide tiles");
  if (c->det) AF_ALLOC(c->d_gtp, sizeof(float) * (size_t)std::max(c->gtp_max, 1LL), "transmit-role sums");
  if (c->nx > 0)  // a slowness grid is set: its per-workgroup partial grids for one chunk
    AF_ALLOC(c->d_gpart, sizeof(float) * (size_t)(c->nx + 3) * (c->nz + 3) * (Pc / af::TILE),
             "partial gradients");
  c->select(0);
  return AF_OK;
}

}  // namespace

void af_ctx::select(int k) {
  const af::Chunk& ch = chunks[k];
  v.t0 = ch.t0;
  v.n_tiles = ch.n_tiles;
  v.p0 = (long long)ch.t0 * TILE;
  v.P = (long long)ch.n_tiles * TILE;
  v.tiles = d_tiles.as<int4>() + ch.t0;
  v.prange = d_prange.as<int2>() + v.p0;
  v.ptxy = d_ptxy.as<float2>() + v.p0;
  v.ptpol = d_ptpol.as<double4>() + v.p0;
  v.tabwork = d_tabwork.as<int2>() + ch.tab_off;
  v.n_tab_work = ch.n_tab;
  v.daswork = d_daswork.as<int2>() + ch.das_off;
  v.n_das_work = ch.n_das;
  v.order = d_order.as<int>() + ch.ord_off;
  v.n_order = ch.n_ord;
  v.wide = d_wide.as<int>() + ch.t0;
  v.n_wide = ch.n_wide;
  v.tbase = d_tbase.as<long long>() + ch.t0;
  const size_t nm = (size_t)n_tiles * ppt;  // slots of one map
  v.map_cmpe = d_maps.as<float>() + (size_t)ch.t0 * ppt;
  v.map_cf = v.map_cmpe + nm;
  v.map_cmcc = v.map_cmpe + 2 * nm;
  v.part = d_part.as<double>() + (size_t)ch.t0 * 4 * (TILE / SUB);  // 4 per sub-tile
  v.gsb = d_gsb.as<float2>() + v.p0;
}

af::Geo af_ctx::geo() const {
  af::Geo g{};
  g.n_elem = N;
  g.ns = Ns;
  g.block = S;
  g.nblk = nb;
  g.nsub = nsub;
  g.n_seg = n_seg;
  g.patch2 = M;
  g.pps = pps;
  g.P = v.P;  // the points of the current view
  g.fs = fs;
  g.fd = fd;
  g.t0 = t0;
  g.t_ttp = t_ttp;
  g.dlens = d_lens;
  g.icl = 1.0 / c_lens;
  g.nsearch = n_search;
  g.flat = flat ? 1 : 0;
  g.nx = nx;
  g.nz = nz;
  g.W = nx + 3;
  g.x0 = (float)x0;
  g.z0 = (float)z0;
  g.idx = (float)(1.0 / dx);
  g.idz = (float)(1.0 / dz);
  return g;
}

extern "C" {

af_status af_create(af_ctx** out, int device, void* stream) {
  if (!out) return AF_ERR_ARG;
  *out = nullptr;
  int n = 0;
  const hipError_t ec = hipGetDeviceCount(&n);
  if (ec != hipSuccess) {
    g_create_err = std::string("af_create: hipGetDeviceCount: ") + hipGetErrorString(ec);
    return AF_ERR_HIP;
  }
  if (device < 0 || device >= n) {
    g_create_err = "af_create: no HIP device " + std::to_string(device);
    return AF_ERR_ARG;
  }
  const hipError_t es = hipSetDevice(device);
  if (es != hipSuccess) {
    g_create_err = std::string("af_create: hipSetDevice: ") + hipGetErrorString(es);
    return AF_ERR_HIP;
  }
  af_ctx* c = new af_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  // address of this device's copy of the no-allocation scratch array (once per
  // device); a failure is reported by the no-allocation call itself
  c->noalloc_ok = af::noalloc_scratch_init(device) == hipSuccess;
  if (c->d_scal.ensure(sizeof(double) * 16) != hipSuccess) {
    delete c;
    return AF_ERR_OOM;
  }
  *out = c;
  return AF_OK;
}

void af_destroy(af_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  delete c;
}

const char* af_last_error(const af_ctx* c) {
  return c ? c->err.c_str() : (g_create_err.empty() ? kNoCtx : g_create_err.c_str());
}

af_status af_set_geometry(af_ctx* c, int n_elem, const double* elem_xz, int n_pix,
                          const double* pix_xz, int patch, double spacing, int n_samples,
                          double fs, double t0, double fd, int block, double fnum, int n_seg) {
  if (!c) return AF_ERR_ARG;
  if (!elem_xz || !pix_xz) return fail(c, AF_ERR_ARG, "af_set_geometry: null array");
  if (n_elem < 3) return fail(c, AF_ERR_ARG, "af_set_geometry: need at least 3 elements");
  if (block <= 0 || n_elem % block != 0 || (block & (block - 1)) != 0 || block > 16)
    return fail(c, AF_ERR_ARG, "af_set_geometry: block must be a power of two <= 16 dividing n_elem");
  if (n_elem / block < 3)
    return fail(c, AF_ERR_ARG, "af_set_geometry: need at least 3 blocks (2 subapertures)");
  if (patch != 1 && patch != 3) return fail(c, AF_ERR_ARG, "af_set_geometry: patch must be 1 or 3");
  if (n_pix <= 0 || n_samples < 2 || !(fs > 0) || n_seg <= 0 || !(fnum > 0) || !(spacing >= 0))
    return fail(c, AF_ERR_ARG, "af_set_geometry: non-positive size or rate");
  AF_HIP(hipSetDevice(c->device), "hipSetDevice");

  c->has_geom = false;
  c->has_grid = false;
  c->N = n_elem;
  c->n_pix = n_pix;
  c->patch = patch;
  c->M = patch * patch;
  c->Ns = n_samples;
  c->fs = fs;
  c->t0 = t0;
  c->fd = fd;
  c->S = block;
  c->nb = n_elem / block;
  c->nsub = c->nb - 1;
  c->fnum = fnum;
  c->n_seg = n_seg;
  c->spacing = spacing;
  const int N = n_elem, M = c->M;
  c->elem_xz.assign(elem_xz, elem_xz + 2 * N);

  // A linear array has every element on one line z = const and a flat lens;
  // otherwise the elements lie on an arc about the origin with a concentric lens.
  double xmax = 0.0, zdev = 0.0;
  for (int a = 0; a < N; ++a) {
    xmax = std::max(xmax, std::fabs(elem_xz[2 * a]));
    zdev = std::max(zdev, std::fabs(elem_xz[2 * a + 1] - elem_xz[1]));
  }
  c->flat = zdev <= 1e-9 * (1.0 + xmax);
  // element geometry: polar (R, sin, cos) on the arc, or (x, z) on the line;
  // elem_pol is the ordering key (polar angle, or x)
  c->elem_R.resize(N);
  c->elem_pol.resize(N);
  std::vector<double4> el(N);
  for (int a = 0; a < N; ++a) {
    const double x = elem_xz[2 * a], z = elem_xz[2 * a + 1];
    const double R = std::sqrt(x * x + z * z);
    c->elem_R[a] = R;
    c->elem_pol[a] = c->flat ? x : std::atan2(x, z);
    el[a] = c->flat ? make_double4(x, z, 0.0, 0.0) : make_double4(R, x / R, z / R, 0.0);
  }
  for (int a = 1; a < N; ++a)
    if (!(c->elem_pol[a] > c->elem_pol[a - 1]))
      return fail(c, AF_ERR_ARG, c->flat ? "af_set_geometry: elements must be ordered by increasing x"
                                         : "af_set_geometry: elements must be ordered by increasing polar angle");
  // element orientation, Eq. 3 (one-sided differences at the two ends)
  std::vector<double> th(N), cth(N), sth(N);
  for (int a = 0; a < N; ++a) {
    const int lo = std::max(a - 1, 0), hi = std::min(a + 1, N - 1);
    th[a] = -std::atan((elem_xz[2 * hi + 1] - elem_xz[2 * lo + 1]) / (elem_xz[2 * hi] - elem_xz[2 * lo]));
    cth[a] = std::cos(th[a]);
    sth[a] = std::sin(th[a]);
  }

  // evaluation points (caller order p = q * M + m)
  const long long P = (long long)n_pix * M;
  c->P = P;
  c->pts_xz.resize(2 * P);
  const int h = patch / 2;
  parallel(host_threads(P), [&](int tid, int nt) {
    const int q0 = (int)((long long)n_pix * tid / nt), q1 = (int)((long long)n_pix * (tid + 1) / nt);
    for (int q = q0; q < q1; ++q)
      for (int m = 0; m < M; ++m) {
        const double ox = (double)(m % patch - h) * spacing, oz = (double)(m / patch - h) * spacing;
        c->pts_xz[2 * ((long long)q * M + m)] = pix_xz[2 * q] + ox;
        c->pts_xz[2 * ((long long)q * M + m) + 1] = pix_xz[2 * q + 1] + oz;
      }
  });

  // active element range of every caller point (Eqs. 2 and 4, FP64).  Small
  // problems scan every element and check that the active set is contiguous;
  // large ones expand from the element nearest in polar angle (on a convex arc
  // the active set is the contiguous run around it).  Split over host threads.
  std::vector<int>& lo_c = c->h_lo;
  std::vector<int>& hi_c = c->h_hi;
  lo_c.resize(P);
  hi_c.resize(P);
  const double half_f = fnum / 2.0;
  auto active = [&](long long p, int a) {
    const double dx = c->pts_xz[2 * p] - elem_xz[2 * a], dz = c->pts_xz[2 * p + 1] - elem_xz[2 * a + 1];
    const double xp = cth[a] * dx - sth[a] * dz;
    const double zp = sth[a] * dx + cth[a] * dz;
    return std::fabs(xp) <= half_f * zp;
  };
  const bool full_scan = (double)P * N <= 2e7;
  std::vector<char> bad_flag(64 * 64, 0);  // one cache line per thread
  auto work = [&](int tid, int nthr) {
    const long long p0 = P * tid / nthr, p1 = P * (tid + 1) / nthr;  // contiguous run
    for (long long p = p0; p < p1; ++p) {
      int lo = N, hi = -1, cnt = 0;
      if (full_scan) {
        for (int a = 0; a < N; ++a)
          if (active(p, a)) {
            lo = std::min(lo, a);
            hi = std::max(hi, a);
            ++cnt;
          }
        if (cnt > 0 && cnt != hi - lo + 1) bad_flag[64 * tid] = 1;
      } else {
        const double ang = c->flat ? c->pts_xz[2 * p] : std::atan2(c->pts_xz[2 * p], c->pts_xz[2 * p + 1]);
        int a0 = (int)(std::upper_bound(c->elem_pol.begin(), c->elem_pol.end(), ang) - c->elem_pol.begin());
        int best = -1;
        for (int a = std::max(a0 - 1, 0); a <= std::min(a0, N - 1); ++a)
          if (active(p, a)) { best = a; break; }
        if (best >= 0) {
          lo = hi = best;
          while (lo > 0 && active(p, lo - 1)) --lo;
          while (hi < N - 1 && active(p, hi + 1)) ++hi;
          cnt = hi - lo + 1;
        }
      }
      lo_c[p] = cnt > 0 ? lo : 1;
      hi_c[p] = cnt > 0 ? hi : 0;
    }
  };
  parallel(std::min(host_threads(P * (full_scan ? N : 8)), 64), work);
  for (char b : bad_flag)
    if (b) return fail(c, AF_ERR_ARG, "af_set_geometry: active elements of a point are not contiguous");

  // spatial tiling of the pixels: k-d partition in (depth, arc length) -- (z, x)
  // for a linear array -- whose
  // splits are multiples of the tile (ppt pixels) and sub-tile (pps pixels)
  // sizes, so every tile and sub-tile is a compact blob
  const int pps = SUB / M;          // whole patches per 64-point sub-tile
  const int ppt = 4 * pps;          // patches per 256-point tile
  c->pps = pps;
  c->ppt = ppt;
  std::vector<double> cu(n_pix), cv(n_pix);
  {
    double rsum = 0;
    for (int q = 0; q < n_pix; ++q) rsum += std::hypot(pix_xz[2 * q], pix_xz[2 * q + 1]);
    const double rref = rsum / n_pix;
    parallel(host_threads(n_pix * 8LL), [&](int tid, int nt) {
      const int q0 = (int)((long long)n_pix * tid / nt), q1 = (int)((long long)n_pix * (tid + 1) / nt);
      for (int q = q0; q < q1; ++q) {
        if (c->flat) {
          cu[q] = pix_xz[2 * q + 1];
          cv[q] = pix_xz[2 * q];
        } else {
          cu[q] = std::hypot(pix_xz[2 * q], pix_xz[2 * q + 1]);
          cv[q] = std::atan2(pix_xz[2 * q], pix_xz[2 * q + 1]) * rref;
        }
      }
    });
  }
  std::vector<int> ord(n_pix);
  std::iota(ord.begin(), ord.end(), 0);
  kd_partition(ord.data(), n_pix, ppt, pps, cu, cv, 4);
  // Pack the pixels, in k-d order, into sub-tiles of pps and tiles of 4 sub-tiles.
  // A tile is closed early (its remaining slots become padding) when the next
  // pixel would widen its span of active blocks beyond what the CMPE kernel
  // stages in LDS, unless the pixel's own span is that wide already (such a tile
  // takes the CMPE stage's device-memory path); with compact images this never
  // happens and the packing follows the k-d units exactly.
  // slot[k] = tile * ppt + sub-tile * pps + s.
  std::vector<long long> slot(n_pix);
  int n_tiles = 0;
  {
    // active block span of every pixel (in parallel), then the greedy packing
    std::vector<int2> pspan(n_pix);
    parallel(host_threads(P), [&](int tid, int nt) {
      const int q0 = (int)((long long)n_pix * tid / nt), q1 = (int)((long long)n_pix * (tid + 1) / nt);
      for (int q = q0; q < q1; ++q) {
        int lo = N, hi = -1;
        for (int m = 0; m < M; ++m) {
          const long long pc = (long long)q * M + m;
          if (lo_c[pc] <= hi_c[pc]) {
            lo = std::min(lo, lo_c[pc] / block);
            hi = std::max(hi, hi_c[pc] / block);
          }
        }
        pspan[q] = make_int2(lo, hi);
      }
    });
    int t = -1, w = 0, sidx = pps, blo = 0, bhi = -1;
    for (int k = 0; k < n_pix; ++k) {
      const int q = ord[k];
      const int plo = pspan[q].x, phi = pspan[q].y;
      bool new_tile = t < 0;
      if (!new_tile && plo <= phi) {
        const int nlo = bhi < blo ? plo : std::min(blo, plo);
        const int nhi = bhi < blo ? phi : std::max(bhi, phi);
        new_tile = nhi - nlo > phi - plo && !af::cmpe_fits_lds(nlo, nhi, c->nsub, pps);
      }
      if (!new_tile && sidx == pps) {  // current sub-tile full: next sub-tile or tile
        if (w == 3) new_tile = true;
        else {
          ++w;
          sidx = 0;
        }
      }
      if (new_tile) {
        ++t;
        w = 0;
        sidx = 0;
        blo = 0;
        bhi = -1;
      }
      if (plo <= phi) {
        const bool empty = bhi < blo;
        blo = empty ? plo : std::min(blo, plo);
        bhi = empty ? phi : std::max(bhi, phi);
      }
      slot[k] = (long long)t * ppt + (long long)w * pps + sidx;
      ++sidx;
    }
    n_tiles = t + 1;
  }
  const long long P_int = (long long)n_tiles * TILE;
  c->n_tiles = n_tiles;
  c->P_int = P_int;
  c->i2c.assign(P_int, -1);
  c->c2i.assign(P, -1);
  for (int k = 0; k < n_pix; ++k) {
    const int q = ord[k];
    const long long tile = slot[k] / ppt;
    const int w = (int)((slot[k] % ppt) / pps), s = (int)((slot[k] % ppt) % pps);
    for (int m = 0; m < M; ++m) {
      const long long pi = tile * TILE + w * SUB + s * M + m;
      c->i2c[pi] = q * M + m;
      c->c2i[(long long)q * M + m] = (int)pi;
    }
  }
  // host staging kept in the context: repeated calls (the dynamic-grid sweep)
  // reuse the pages instead of faulting in fresh ones
  std::vector<double4>& ptpol = c->h_ptpol;
  std::vector<float2>& ptxy = c->h_ptxy;
  std::vector<int2>& prange = c->h_prange;
  ptpol.resize(P_int);
  ptxy.resize(P_int);
  prange.resize(P_int);
  c->tile_lo.assign(n_tiles, N);
  c->tile_hi.assign(n_tiles, -1);
  {
    // contiguous runs of whole tiles per thread
    const int nthr = host_threads(P_int);
    std::vector<long long> pairs(nthr * 8, 0), samples(nthr * 8, 0);  // one cache line apart
    parallel(nthr, [&](int tid, int nt) {
      const int t0 = (int)((long long)n_tiles * tid / nt), t1 = (int)((long long)n_tiles * (tid + 1) / nt);
      long long np = 0, ns = 0;
      for (int t = t0; t < t1; ++t) {
        int tlo = N, thi = -1;
        for (long long pi = (long long)t * TILE; pi < (long long)(t + 1) * TILE; ++pi) {
          const int pc = c->i2c[pi];
          const long long src = pc >= 0 ? pc : c->i2c[(long long)t * TILE];
          const double x = c->pts_xz[2 * src], z = c->pts_xz[2 * src + 1];
          const double rho = std::sqrt(x * x + z * z);
          ptpol[pi] = c->flat ? make_double4(x, z, 0.0, 0.0) : make_double4(rho, x / rho, z / rho, 0.0);
          ptxy[pi] = make_float2((float)x, (float)z);
          int lo = 1, hi = 0;
          if (pc >= 0) {
            lo = lo_c[pc];
            hi = hi_c[pc];
          }
          prange[pi] = make_int2(lo, hi);
          if (lo <= hi) {
            tlo = std::min(tlo, lo);
            thi = std::max(thi, hi);
            np += hi - lo + 1;
            ns += (long long)(hi - lo + 1) * (hi - lo + 1);
          }
        }
        c->tile_lo[t] = tlo;
        c->tile_hi[t] = thi;
      }
      pairs[tid * 8] = np;
      samples[tid * 8] = ns;
    });
    c->active_pairs = 0;
    c->active_samples = 0;
    for (int t = 0; t < nthr; ++t) {
      c->active_pairs += pairs[t * 8];
      c->active_samples += samples[t * 8];
    }
  }
  af_status st;
  // element frames (position and the orientation of Eq. 3) for the dynamic grid
  c->elem_frame.resize(N);
  for (int a = 0; a < N; ++a)
    c->elem_frame[a] = make_double4(elem_xz[2 * a], elem_xz[2 * a + 1], cth[a], sth[a]);
  c->pix_xz.assign(pix_xz, pix_xz + 2 * (size_t)n_pix);
  c->dyn_on = false;
  if ((st = upload(c, c->d_elem, el, "elements")) != AF_OK) return st;
  if ((st = upload(c, c->d_ptpol, ptpol, "points")) != AF_OK) return st;
  if ((st = upload(c, c->d_ptxy, ptxy, "points")) != AF_OK) return st;
  if ((st = upload(c, c->d_prange, prange, "point ranges")) != AF_OK) return st;
  if ((st = upload(c, c->d_c2i, c->c2i, "point map")) != AF_OK) return st;
  if ((st = upload(c, c->d_i2c, c->i2c, "point map")) != AF_OK) return st;

  AF_ALLOC(c->d_gsb, sizeof(float2) * (size_t)P_int, "brightness gradient");
  AF_ALLOC(c->d_part, sizeof(double) * 4 * (size_t)(P_int / SUB), "partials");
  AF_ALLOC(c->d_maps, sizeof(float) * 3 * (size_t)n_tiles * ppt, "maps");
  if ((st = build_work_lists(c)) != AF_OK) return st;  // chunks and their buffers
  c->has_geom = true;
  return AF_OK;
}

af_status af_set_lens(af_ctx* c, double d_lens, double c_lens, double t_ttp, int mode,
                      double c_ref) {
  if (!c) return AF_ERR_ARG;
  if (!(d_lens >= 0) || !(c_lens > 0) || !std::isfinite(t_ttp) || !std::isfinite(d_lens) ||
      !std::isfinite(c_lens))
    return fail(c, AF_ERR_ARG, "af_set_lens: need d_lens >= 0, c_lens > 0, finite t_ttp");
  if (mode != AF_LENS_BENT && mode != AF_LENS_CONVENTIONAL && mode != AF_LENS_NONE)
    return fail(c, AF_ERR_ARG, "af_set_lens: unknown lens mode");
  if (mode == AF_LENS_CONVENTIONAL && !(c_ref > 0 && std::isfinite(c_ref)))
    return fail(c, AF_ERR_ARG, "af_set_lens: the conventional model needs c_ref > 0");
  c->lens_mode = mode;
  c->d_lens_phys = d_lens;
  c->t_ttp_phys = t_ttp;
  c->c_lens = c_lens;
  c->c_ref = mode == AF_LENS_CONVENTIONAL ? c_ref : 1.54;
  // the bent-ray model traces the lens (Eqs. 7-8); the straight-ray models start
  // their rays at the elements, the conventional one adding the scalar lens
  // offset of Eq. 6 (round trip through the lens along the normal at c_lens
  // instead of c_ref) to the time-to-peak constant
  c->d_lens = mode == AF_LENS_BENT ? d_lens : 0.0;
  c->t_ttp = t_ttp;
  if (mode == AF_LENS_CONVENTIONAL) c->t_ttp += 2.0 * d_lens * (1.0 / c_lens - 1.0 / c_ref);
  c->has_lens = true;
  c->has_grid = false;
  return AF_OK;
}

af_status af_set_refraction_search(af_ctx* c, int n_search) {
  if (!c) return AF_ERR_ARG;
  if (n_search != 0 && (n_search < 2 || n_search > AF_MAX_SEARCH))
    return fail(c, AF_ERR_ARG, "af_set_refraction_search: n_search must be 0 or in [2, 4096]");
  c->n_search = n_search;
  return AF_OK;
}

af_status af_set_deterministic(af_ctx* c, int on) {
  if (!c) return AF_ERR_ARG;
  if (on != 0 && on != 1) return fail(c, AF_ERR_ARG, "af_set_deterministic: on must be 0 or 1");
  c->det = on != 0;
  if (!c->has_geom) return AF_OK;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AF_ERR_HIP, "hipSetDevice");
  // under a memory budget the slabs count towards it: the chunks are cut again
  if (c->mem_budget > 0) return build_work_lists(c);
  if (c->det) AF_ALLOC(c->d_gtp, sizeof(float) * (size_t)std::max(c->gtp_max, 1LL), "transmit-role sums");
  return AF_OK;
}

af_status af_set_memory_budget(af_ctx* c, size_t bytes) {
  if (!c) return AF_ERR_ARG;
  c->mem_budget = bytes;
  if (!c->has_geom) return AF_OK;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AF_ERR_HIP, "hipSetDevice");
  AF_HIP(hipStreamSynchronize(c->stream), "af_set_memory_budget");
  // free the chunk-sized buffers so that a smaller chunk really holds less memory
  for (af::DBuf* b : {&c->d_tab, &c->d_ray_uv, &c->d_ray_l2, &c->d_bblk, &c->d_gT, &c->d_gtp,
                      &c->d_cmpe_wide, &c->d_gsum, &c->d_chan})
    b->release();
  return build_work_lists(c);
}

af_status af_set_slowness(af_ctx* c, int nx, int nz, double x0, double z0, double dx, double dz,
                          const float* s_dev) {
  if (!c) return AF_ERR_ARG;
  if (!c->has_geom || !c->has_lens)
    return fail(c, AF_ERR_STATE, "af_set_slowness: set geometry and lens first");
  if (nx < 2 || nz < 2 || !(dx > 0) || !(dz > 0) || !s_dev)
    return fail(c, AF_ERR_ARG, "af_set_slowness: bad grid");
  // the path adjoint keeps four copies of the padded grid in LDS (160 KB per
  // workgroup)
  if ((size_t)(nx + 3) * (nz + 3) > 9600)
    return fail(c, AF_ERR_ARG, "af_set_slowness: grid larger than (nx+3)(nz+3) <= 9600 nodes");
  const double x1 = x0 + (nx - 1) * dx, z1 = z0 + (nz - 1) * dz, tol = 1e-9;
  auto inside = [&](double x, double z) {
    return x >= x0 - tol && x <= x1 + tol && z >= z0 - tol && z <= z1 + tol;
  };
  double amin = 1e300, amax = -1e300;
  for (int a = 0; a < c->N; ++a) {
    amin = std::min(amin, c->elem_pol[a]);
    amax = std::max(amax, c->elem_pol[a]);
  }
  if (c->dyn_on) {
    // dynamic grid: the box and angle range of every point at every speed of the sweep
    if (!inside(c->dyn_box[0], c->dyn_box[2]) || !inside(c->dyn_box[1], c->dyn_box[3]))
      return fail(c, AF_ERR_ARG, "af_set_slowness: grid does not cover every point of the dynamic grid");
    amin = std::min(amin, c->dyn_ang[0]);
    amax = std::max(amax, c->dyn_ang[1]);
  } else {
    const int nthr = host_threads(c->P);
    std::vector<double> tmin(nthr * 8, 1e300), tmax(nthr * 8, -1e300);  // one cache line apart
    std::vector<long long> out(nthr * 8, 0);
    parallel(nthr, [&](int tid, int nt) {
      const long long p0 = c->P * tid / nt, p1 = c->P * (tid + 1) / nt;
      double lo = 1e300, hi = -1e300;
      long long bad = 0;
      for (long long p = p0; p < p1; ++p) {
        const double x = c->pts_xz[2 * p], z = c->pts_xz[2 * p + 1];
        bad += inside(x, z) ? 0 : 1;
        const double ang = c->flat ? x : std::atan2(x, z);
        lo = std::min(lo, ang);
        hi = std::max(hi, ang);
      }
      tmin[tid * 8] = lo;
      tmax[tid * 8] = hi;
      out[tid * 8] = bad;
    });
    for (int t = 0; t < nthr; ++t) {
      if (out[t * 8]) return fail(c, AF_ERR_ARG, "af_set_slowness: grid does not cover every point");
      amin = std::min(amin, tmin[t * 8]);
      amax = std::max(amax, tmax[t * 8]);
    }
  }
  // flat lens: the plane segment over [amin, amax] in x (its two ends)
  for (int a = 0; c->flat && a < c->N; ++a) {
    const double zl = c->elem_xz[2 * a + 1] + c->d_lens;
    if (!inside(amin, zl) || !inside(amax, zl))
      return fail(c, AF_ERR_ARG, "af_set_slowness: grid does not cover the lens surface");
  }
  // lens arc over [amin, amax] (both ends and the apex if it is inside)
  for (int a = 0; !c->flat && a < c->N; ++a) {
    const double RL = c->elem_R[a] + c->d_lens;
    const double cand[3] = {amin, amax, 0.0};
    for (int k = 0; k < 3; ++k) {
      if (k == 2 && !(amin <= 0.0 && amax >= 0.0)) continue;
      if (!inside(RL * std::sin(cand[k]), RL * std::cos(cand[k])))
        return fail(c, AF_ERR_ARG, "af_set_slowness: grid does not cover the lens arc");
    }
  }
  c->nx = nx;
  c->nz = nz;
  c->x0 = x0;
  c->z0 = z0;
  c->dx = dx;
  c->dz = dz;
  const size_t n = (size_t)nx * nz, np = (size_t)(nx + 3) * (nz + 3);
  AF_ALLOC(c->d_s, sizeof(float) * n, "slowness");
  AF_ALLOC(c->d_regg, sizeof(float) * n, "regulariser gradient");
  AF_ALLOC(c->d_grad, sizeof(float) * n, "gradient");
  AF_ALLOC(c->d_gdev, sizeof(float) * np, "deviation grid");
  AF_ALLOC(c->d_gpad, sizeof(float) * np, "padded gradient");
  // one partial grid per tile of a chunk that has work (at most every tile of the
  // chunk: the dynamic grid may give more tiles work than the layout of
  // af_set_geometry)
  AF_ALLOC(c->d_gpart, sizeof(float) * np * std::max(c->P_chunk / TILE, 1LL), "partial gradients");
  AF_ALLOC(c->d_terms, sizeof(float) * 8, "terms");
  c->has_grid = false;  // until the new values have passed the check
  AF_HIP(hipMemcpyAsync(c->d_s.p, s_dev, sizeof(float) * n, hipMemcpyDeviceToDevice, c->stream),
         "af_set_slowness copy");
  af_status st = check_slowness(c, c->d_s.as<float>(), n, "af_set_slowness");
  if (st != AF_OK) return st;
  c->has_grid = true;
  return AF_OK;
}

}  // extern "C"

namespace {

af_status ready(af_ctx* c, const void* iq) {
  if (!c) return AF_ERR_ARG;
  if (!c->has_geom || !c->has_lens || !c->has_grid)
    return fail(c, AF_ERR_STATE, "af: set geometry, lens and slowness first");
  if (!iq) return fail(c, AF_ERR_ARG, "af: null channel data");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AF_ERR_HIP, "hipSetDevice");
  return AF_OK;
}

// grid prep: c_med, the deviation grid, the regulariser (with lp)
af_status run_prepare(af_ctx* c, const af_loss_params* lp) {
  AF_KERNEL(AF_K_PREPARE,
            af::launch_prepare_grid(c, c->d_s.as<float>(), c->nx, c->nz, c->d_gdev.as<float>(),
                                    c->d_scal.as<double>(), lp ? 1 : 0, lp, c->d_regg.as<float>()),
            "prepare_grid");
  return AF_OK;
}

// Table, block images and CMPE stage of the current view; with write_g the
// unscaled dL/dB^blk goes to gout (or in place into the block images).
af_status run_view_forward(af_ctx* c, const float2* iq, const af_loss_params* lp, bool write_g,
                           float2* gout) {
  AF_KERNEL(AF_K_TABLE, af::launch_table(c), "table");
  AF_KERNEL(AF_K_DAS_FWD, af::launch_das_fwd(c, iq, c->d_bblk.as<float2>()), "das_fwd");
  const float sb_scale = (float)(-2.0 * lp->w_sb / ((double)lp->sb_ref * c->n_pix));
  float2* g = gout ? gout : c->d_bblk.as<float2>();
  AF_KERNEL(AF_K_CMPE,
            af::launch_cmpe(c, c->d_bblk.as<float2>(), g, write_g ? 1 : 0, lp->rho_thresh,
                            sb_scale, c->v.map_cmpe, c->v.map_cf, c->v.map_cmcc, nullptr),
            "cmpe");
  return AF_OK;
}

// Adjoint of the current view's forward (dL/dB^blk in gblk, scaled: final, else
// scaled on the fly from the terms of finalize): its grid sums into out [nodes].
af_status run_view_backward(af_ctx* c, const float2* iq, const float2* gblk, bool scaled,
                            float* out) {
  AF_KERNEL(AF_K_DAS_ADJ, af::launch_das_adj(c, iq, gblk, scaled), "das_adj");
  AF_KERNEL(AF_K_PATH_ADJ, af::launch_path_adj(c, out), "path_adj");
  return AF_OK;
}

// The objective (terms) and, with grad, its gradient with respect to the slowness.
// One chunk: forward and adjoint on the same table.  Several chunks (bounded
// memory): a forward pass over the chunks gives the terms (the CMPE mean needs
// every chunk's valid pairs); the adjoint pass then recomputes each chunk's table
// and block images instead of keeping them, and the chunks' grid sums are added
// in chunk order.
af_status run_loss(af_ctx* c, const af_complex* iq, const af_loss_params* lp, float* terms,
                   float* grad) {
  const float2* iqf = reinterpret_cast<const float2*>(iq);
  af_status st = run_prepare(c, lp);
  if (st != AF_OK) return st;
  const int K = (int)c->chunks.size();
  const bool g = grad != nullptr;
  for (int k = 0; k < K; ++k) {
    c->select(k);
    if ((st = run_view_forward(c, iqf, lp, g && K == 1, nullptr)) != AF_OK) return st;
  }
  AF_KERNEL(AF_K_FINALIZE, af::launch_finalize(c, lp, terms), "finalize");
  c->rho_last = lp->rho_thresh;
  if (!g) return AF_OK;
  if (K == 1) {
    if ((st = run_view_backward(c, iqf, c->d_bblk.as<float2>(), false, c->d_gpad.as<float>())) != AF_OK)
      return st;
  } else {
    const size_t nodes = (size_t)(c->nx + 3) * (c->nz + 3);
    AF_ALLOC(c->d_gsum, sizeof(float) * nodes * K, "chunk grid sums");
    for (int k = 0; k < K; ++k) {
      c->select(k);
      if ((st = run_view_forward(c, iqf, lp, true, nullptr)) != AF_OK) return st;
      if ((st = run_view_backward(c, iqf, c->d_bblk.as<float2>(), false,
                                  c->d_gsum.as<float>() + nodes * k)) != AF_OK)
        return st;
    }
    AF_HIP(af::launch_sum_grids(c, c->d_gsum.as<float>(), K, c->d_gpad.as<float>()), "chunk sums");
  }
  AF_KERNEL(AF_K_FOLD, af::launch_grad_fold(c, grad), "grad_fold");
  return AF_OK;
}

// The calls that hand the whole [nb][nb][P] block-image gradient, or the receive
// channel images of every point, to or from the caller need every point at once.
af_status need_unbounded(af_ctx* c, const char* who) {
  if (c->bounded())
    return fail(c, AF_ERR_STATE, std::string(who) + ": not available under a memory budget");
  c->select(0);
  return AF_OK;
}

af_status check_lp(af_ctx* c, const af_loss_params* lp) {
  if (!lp) return fail(c, AF_ERR_ARG, "af: null loss parameters");
  if (!(lp->sb_ref > 0)) return fail(c, AF_ERR_ARG, "af: sb_ref must be > 0");
  return AF_OK;
}

// The physical lens surface the dynamic grid measures depth from: the radius of
// the concentric arc, or the z of the flat lens plane.
double dyn_lens_surface(const af_ctx* c) {
  return c->flat ? c->elem_xz[1] + c->d_lens_phys : c->elem_R[0] + c->d_lens_phys;
}

// Caller point p of the dynamic grid at relative speed k = c_g / c_ref with patch
// spacing sp (host; the device does the same in k_sweep_points): the pixel's
// depth below the lens surface scaled by k along its polar angle (arc) or straight
// down (line), then the patch offset.
void dyn_point(const af_ctx* c, double rl, double k, double sp, long long p, double& x,
               double& z) {
  const int q = (int)(p / c->M), m = (int)(p % c->M), h = c->patch / 2;
  const double cx = c->pix_xz[2 * (size_t)q], cz = c->pix_xz[2 * (size_t)q + 1];
  if (c->flat) {
    x = cx;
    z = rl + (cz - rl) * k;
  } else {
    const double rho = std::sqrt(cx * cx + cz * cz);
    const double f = (rl + (rho - rl) * k) / rho;
    x = cx * f;
    z = cz * f;
  }
  x += (double)(m % c->patch - h) * sp;
  z += (double)(m / c->patch - h) * sp;
}

// Moves the points of the dynamic grid to speed c_g on the device, reads the
// tiles' active element ranges back (the stream is synchronised) and rebuilds
// the work lists from them.  A failure leaves the context without geometry.
af_status move_points(af_ctx* c, double c_g, const char* who) {
  c->has_geom = false;
  AF_HIP(af::launch_sweep_points(c, c_g / c->dyn_cref, c_g / (2.0 * c->dyn_fc),
                                 dyn_lens_surface(c), c->d_tstat.as<af::TileStat>()),
         who);
  std::vector<af::TileStat> ts(c->n_tiles);
  AF_HIP(hipMemcpyAsync(ts.data(), c->d_tstat.p, sizeof(af::TileStat) * ts.size(),
                        hipMemcpyDeviceToHost, c->stream),
         who);
  AF_HIP(hipStreamSynchronize(c->stream), who);
  c->active_pairs = 0;
  c->active_samples = 0;
  for (int t = 0; t < c->n_tiles; ++t) {
    if (ts[t].bad)
      return fail(c, AF_ERR_ARG, std::string(who) + ": active elements of a point are not contiguous");
    c->tile_lo[t] = ts[t].lo;
    c->tile_hi[t] = ts[t].hi;
    c->active_pairs += ts[t].pairs;
    c->active_samples += ts[t].samples;
  }
  af_status st = build_work_lists(c);
  if (st != AF_OK) return st;
  c->spacing = c_g / (2.0 * c->dyn_fc);
  c->dyn_c = c_g;
  c->has_geom = true;
  return AF_OK;
}

}  // namespace

extern "C" {

af_status af_beamform(af_ctx* c, const af_complex* iq, af_complex* blk, af_complex* img,
                      float* maps) {
  af_status st = ready(c, iq);
  if (st != AF_OK) return st;
  if ((st = run_prepare(c, nullptr)) != AF_OK) return st;
  const float2* iqf = reinterpret_cast<const float2*>(iq);
  for (int k = 0; k < (int)c->chunks.size(); ++k) {
    c->select(k);
    AF_KERNEL(AF_K_TABLE, af::launch_table(c), "table");
    AF_HIP(af::launch_das_fwd(c, iqf, c->d_bblk.as<float2>()), "das_fwd");
    if (maps)
      AF_HIP(af::launch_cmpe(c, c->d_bblk.as<float2>(), nullptr, 0, c->rho_last, 0.f,
                             c->v.map_cmpe, c->v.map_cf, c->v.map_cmcc, nullptr),
             "cmpe maps");
    if (blk || img || maps)
      AF_HIP(af::launch_export_images(c, c->d_bblk.as<float2>(), reinterpret_cast<float2*>(blk),
                                      reinterpret_cast<float2*>(img), maps),
             "export images");
  }
  return AF_OK;
}

static af_status channel_images(af_ctx* c, const af_complex* iq) {
  af_status st = ready(c, iq);
  if (st != AF_OK) return st;
  if ((st = need_unbounded(c, "af_channel_images / af_lag_one_coherence")) != AF_OK) return st;
  if ((st = run_prepare(c, nullptr)) != AF_OK) return st;
  AF_KERNEL(AF_K_TABLE, af::launch_table(c), "table");
  AF_ALLOC(c->d_chan, sizeof(float2) * (size_t)c->N * c->P_int, "channel images");
  AF_HIP(af::launch_channel_images(c, reinterpret_cast<const float2*>(iq), c->d_chan.as<float2>()),
         "channel images");
  return AF_OK;
}

af_status af_channel_images(af_ctx* c, const af_complex* iq, af_complex* x) {
  if (c && !x) return fail(c, AF_ERR_ARG, "af_channel_images: null output");
  af_status st = channel_images(c, iq);
  if (st != AF_OK) return st;
  AF_HIP(af::launch_export_rx(c, c->d_chan.as<float2>(), reinterpret_cast<float2*>(x)),
         "export channel images");
  return AF_OK;
}

af_status af_lag_one_coherence(af_ctx* c, const af_complex* iq, float* loc) {
  if (c && !loc) return fail(c, AF_ERR_ARG, "af_lag_one_coherence: null output");
  af_status st = channel_images(c, iq);
  if (st != AF_OK) return st;
  AF_HIP(af::launch_loc(c, c->d_chan.as<float2>(), loc), "lag-one coherence");
  return AF_OK;
}

af_status af_loss_and_grad(af_ctx* c, const af_complex* iq, const af_loss_params* lp, float* terms,
                           float* grad) {
  af_status st = ready(c, iq);
  if (st != AF_OK) return st;
  if ((st = check_lp(c, lp)) != AF_OK) return st;
  if (!terms) return fail(c, AF_ERR_ARG, "af_loss_and_grad: null terms");
  return run_loss(c, iq, lp, terms, grad);
}

af_status af_forward(af_ctx* c, const af_complex* iq, const af_loss_params* lp, float* terms,
                     af_complex* gblk) {
  af_status st = ready(c, iq);
  if (st != AF_OK) return st;
  if ((st = check_lp(c, lp)) != AF_OK) return st;
  if (!terms || !gblk) return fail(c, AF_ERR_ARG, "af_forward: null output");
  if ((st = need_unbounded(c, "af_forward")) != AF_OK) return st;
  if ((st = run_prepare(c, lp)) != AF_OK) return st;
  float2* g = reinterpret_cast<float2*>(gblk);
  if ((st = run_view_forward(c, reinterpret_cast<const float2*>(iq), lp, true, g)) != AF_OK)
    return st;
  AF_KERNEL(AF_K_FINALIZE, af::launch_finalize(c, lp, terms), "finalize");
  AF_KERNEL(AF_K_GSCALE, af::launch_gscale(c, g), "gscale");  // the final scale, for the caller
  c->rho_last = lp->rho_thresh;
  return AF_OK;
}

af_status af_backward(af_ctx* c, const af_complex* iq, const af_loss_params* lp,
                      const af_complex* gblk, float* grad) {
  af_status st = ready(c, iq);
  if (st != AF_OK) return st;
  if ((st = check_lp(c, lp)) != AF_OK) return st;
  if (!gblk || !grad) return fail(c, AF_ERR_ARG, "af_backward: null buffer");
  if ((st = need_unbounded(c, "af_backward")) != AF_OK) return st;
  // recompute: no table is kept between calls
  if ((st = run_prepare(c, lp)) != AF_OK) return st;
  AF_KERNEL(AF_K_TABLE, af::launch_table(c), "table");
  if ((st = run_view_backward(c, reinterpret_cast<const float2*>(iq),
                              reinterpret_cast<const float2*>(gblk), true,
                              c->d_gpad.as<float>())) != AF_OK)
    return st;
  AF_KERNEL(AF_K_FOLD, af::launch_grad_fold(c, grad), "grad_fold");
  return AF_OK;
}

af_status af_autofocus_step(af_ctx* c, const af_complex* iq, const af_loss_params* lp,
                            const af_adam_params* ap, int step, float* s, float* m, float* v,
                            float* terms) {
  af_status st = ready(c, iq);
  if (st != AF_OK) return st;
  if (!ap || !s || !m || !v || !terms || step < 1)
    return fail(c, AF_ERR_ARG, "af_autofocus_step: bad argument");
  if ((st = check_lp(c, lp)) != AF_OK) return st;
  const size_t n = (size_t)c->nx * c->nz;
  AF_HIP(hipMemcpyAsync(c->d_s.p, s, sizeof(float) * n, hipMemcpyDeviceToDevice, c->stream), "copy s");
  if ((st = run_loss(c, iq, lp, terms, c->d_grad.as<float>())) != AF_OK) return st;
  AF_KERNEL(AF_K_ADAM, af::launch_adam(c, ap, step, s, m, v, c->d_grad.as<float>()), "adam");
  return AF_OK;
}

af_status af_set_dynamic_grid(af_ctx* c, double c_ref, double fc, double c_min, double c_max) {
  if (!c) return AF_ERR_ARG;
  if (!c->has_geom || !c->has_lens)
    return fail(c, AF_ERR_STATE, "af_set_dynamic_grid: set geometry and lens first");
  if (!(c_ref > 0) || !(fc > 0) || !(c_min > 0) || !(c_max >= c_min) || !std::isfinite(c_max) ||
      !std::isfinite(c_ref) || !std::isfinite(fc))
    return fail(c, AF_ERR_ARG, "af_set_dynamic_grid: need c_ref, fc > 0 and 0 < c_min <= c_max");
  AF_HIP(hipSetDevice(c->device), "hipSetDevice");
  const double rl = dyn_lens_surface(c);
  // per internal point: its pixel centre and patch offset (units of the spacing);
  // a padding slot repeats the first point of its tile, as in the geometry set-up
  const int M = c->M, h = c->patch / 2;
  std::vector<double4> base(c->P_int);
  for (long long pi = 0; pi < c->P_int; ++pi) {
    int pc = c->i2c[pi];
    if (pc < 0) pc = c->i2c[(pi / TILE) * TILE];
    const int q = pc / M, m = pc % M;
    base[pi] = make_double4(c->pix_xz[2 * (size_t)q], c->pix_xz[2 * (size_t)q + 1],
                            (double)(m % c->patch - h), (double)(m / c->patch - h));
  }
  // every point moves on a straight line as the speed changes (its position is
  // affine in c_g), so the points at c_min and c_max bound the box and the polar
  // angles (monotone along a line that misses the origin) of every speed
  double box[4] = {1e300, -1e300, 1e300, -1e300}, ang[2] = {1e300, -1e300};
  for (double cg : {c_min, c_max}) {
    const double k = cg / c_ref, sp = cg / (2.0 * fc);
    for (long long p = 0; p < c->P; ++p) {
      double x, z;
      dyn_point(c, rl, k, sp, p, x, z);
      box[0] = std::min(box[0], x);
      box[1] = std::max(box[1], x);
      box[2] = std::min(box[2], z);
      box[3] = std::max(box[3], z);
      const double a = c->flat ? x : std::atan2(x, z);
      ang[0] = std::min(ang[0], a);
      ang[1] = std::max(ang[1], a);
    }
  }
  af_status st;
  if ((st = upload(c, c->d_dyn_base, base, "dynamic grid")) != AF_OK) return st;
  if ((st = upload(c, c->d_elemf, c->elem_frame, "element frames")) != AF_OK) return st;
  AF_ALLOC(c->d_tstat, sizeof(af::TileStat) * (size_t)std::max(c->n_tiles, 1), "tile statistics");
  c->dyn_on = true;
  c->dyn_cref = c_ref;
  c->dyn_fc = fc;
  c->dyn_cmin = c_min;
  c->dyn_cmax = c_max;
  c->dyn_c = 0.0;  // the points are still those of af_set_geometry
  std::copy(box, box + 4, c->dyn_box);
  std::copy(ang, ang + 2, c->dyn_ang);
  c->has_grid = false;  // the slowness grid must now cover every speed of the sweep
  return AF_OK;
}

af_status af_set_sweep_speed(af_ctx* c, double c_g) {
  if (!c) return AF_ERR_ARG;
  if (!c->dyn_on) return fail(c, AF_ERR_STATE, "af_set_sweep_speed: no dynamic grid");
  if (!(c_g >= c->dyn_cmin * (1.0 - 1e-12) && c_g <= c->dyn_cmax * (1.0 + 1e-12)))
    return fail(c, AF_ERR_ARG, "af_set_sweep_speed: speed outside the dynamic grid's range");
  AF_HIP(hipSetDevice(c->device), "hipSetDevice");
  return move_points(c, c_g, "af_set_sweep_speed");
}

af_status af_sweep(af_ctx* c, const af_complex* iq, const af_loss_params* lp, int n,
                   const double* speeds, int dynamic, double static_c, float* cmpe_dev,
                   double* best) {
  af_status st = ready(c, iq);
  if (st != AF_OK) return st;
  if ((st = check_lp(c, lp)) != AF_OK) return st;
  if (!c->dyn_on) return fail(c, AF_ERR_STATE, "af_sweep: no dynamic grid");
  if (n < 1 || !speeds || !cmpe_dev || !best) return fail(c, AF_ERR_ARG, "af_sweep: bad argument");
  auto in_range = [&](double v) {
    return v >= c->dyn_cmin * (1.0 - 1e-12) && v <= c->dyn_cmax * (1.0 + 1e-12);
  };
  for (int k = 0; k < n; ++k)
    if (!in_range(speeds[k])) return fail(c, AF_ERR_ARG, "af_sweep: speed outside the dynamic grid's range");
  if (!dynamic && !in_range(static_c))
    return fail(c, AF_ERR_ARG, "af_sweep: static speed outside the dynamic grid's range");
  const int ns = c->nx * c->nz;
  if (!dynamic && (st = move_points(c, static_c, "af_sweep")) != AF_OK) return st;
  for (int k = 0; k < n; ++k) {
    if (dynamic && (st = move_points(c, speeds[k], "af_sweep")) != AF_OK) return st;
    AF_HIP(af::launch_fill(c, c->d_s.as<float>(), ns, (float)(1.0 / speeds[k])), "uniform slowness");
    if ((st = run_loss(c, iq, lp, c->d_terms.as<float>(), nullptr)) != AF_OK) return st;
    AF_HIP(hipMemcpyAsync(cmpe_dev + k, c->d_terms.as<float>() + AF_TERM_CMPE, sizeof(float),
                          hipMemcpyDeviceToDevice, c->stream),
           "af_sweep copy");
  }
  std::vector<float> v(n);
  AF_HIP(hipMemcpyAsync(v.data(), cmpe_dev, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream),
         "af_sweep read-back");
  AF_HIP(hipStreamSynchronize(c->stream), "af_sweep read-back");
  int kb = 0;  // the lowest CMPE, the first one on ties
  for (int k = 1; k < n; ++k)
    if (v[k] < v[kb]) kb = k;
  *best = speeds[kb];
  if (dynamic && (st = move_points(c, speeds[kb], "af_sweep")) != AF_OK) return st;
  AF_HIP(af::launch_fill(c, c->d_s.as<float>(), ns, (float)(1.0 / speeds[kb])), "uniform slowness");
  return AF_OK;
}

af_status af_travel_times(af_ctx* c, float* t_dev) {
  af_status st = ready(c, t_dev);
  if (st != AF_OK) return st;
  if ((st = run_prepare(c, nullptr)) != AF_OK) return st;
  for (int k = 0; k < (int)c->chunks.size(); ++k) {
    c->select(k);
    AF_KERNEL(AF_K_TABLE, af::launch_table(c), "table");
    AF_HIP(af::launch_export_T(c, t_dev), "export T");
  }
  return AF_OK;
}

af_status af_simulate(af_ctx* c, int n_scat, const double* scat_xz, const float* amp, int nx, int nz,
                      double x0, double z0, double dx, double dz, const float* s_true, int n_seg,
                      double fc, double frac_bw, af_complex* iq) {
  if (!c) return AF_ERR_ARG;
  if (!c->has_geom || !c->has_lens) return fail(c, AF_ERR_STATE, "af_simulate: set geometry and lens first");
  if (n_scat <= 0 || !scat_xz || !amp || !s_true || !iq || nx < 2 || nz < 2 || n_seg <= 0 ||
      !(fc > 0) || !(frac_bw > 0) || !(dx > 0) || !(dz > 0))
    return fail(c, AF_ERR_ARG, "af_simulate: bad argument");
  const double x1 = x0 + (nx - 1) * dx, z1 = z0 + (nz - 1) * dz;
  for (int k = 0; k < n_scat; ++k) {
    const double x = scat_xz[2 * k], z = scat_xz[2 * k + 1];
    if (!(x >= x0 && x <= x1 && z >= z0 && z <= z1))
      return fail(c, AF_ERR_ARG, "af_simulate: grid does not cover every scatterer");
  }
  if ((size_t)2 * c->Ns * sizeof(unsigned long long) > 160 * 1024)
    return fail(c, AF_ERR_ARG, "af_simulate: records longer than 10240 samples");
  // the fixed-point record holds sums of magnitude below 2^31; the envelope is at
  // most 1, so the sum of |amp| bounds every sample
  double amp_sum = 0.0;
  for (int k = 0; k < n_scat; ++k) amp_sum += std::fabs((double)amp[k]);
  if (!(amp_sum < 2147483648.0))
    return fail(c, AF_ERR_ARG, "af_simulate: amplitudes not finite or their sum not below 2^31");
  AF_HIP(hipSetDevice(c->device), "hipSetDevice");
  af_status st = check_slowness(c, s_true, (size_t)nx * nz, "af_simulate");
  if (st != AF_OK) return st;
  AF_HIP(af::launch_simulate(c, n_scat, scat_xz, amp, nx, nz, x0, z0, dx, dz, s_true, n_seg, fc,
                             frac_bw, reinterpret_cast<float2*>(iq)),
         "simulate");
  return AF_OK;
}

static af_status conv_args(af_ctx* c, int B, int H, int W, int Cin, int Cout, int stride) {
  if (!c) return AF_ERR_ARG;
  if (B <= 0 || H <= 0 || W <= 0 || Cin < 1 || Cin > 32 || Cout < 1 || Cout > 32 ||
      (stride != 1 && stride != 2))
    return fail(c, AF_ERR_ARG, "af_conv3x3: need 1 <= Cin, Cout <= 32, stride 1 or 2, positive sizes");
  if ((long long)B * H * W * std::max(Cin, Cout) * 2 >= (1LL << 31))
    return fail(c, AF_ERR_ARG, "af_conv3x3: activations of 2 GiB or more");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, AF_ERR_HIP, "hipSetDevice");
  return AF_OK;
}

af_status af_conv3x3_pack(af_ctx* c, int Cin, int Cout, const float* w, void* wpack, void* wtpack) {
  af_status st = conv_args(c, 1, 1, 1, Cin, Cout, 1);
  if (st != AF_OK) return st;
  if (!w || !wpack) return fail(c, AF_ERR_ARG, "af_conv3x3_pack: null pointer");
  AF_HIP(af::launch_conv_pack(c, Cin, Cout, w, wpack, wtpack), "conv pack");
  return AF_OK;
}

af_status af_conv3x3_fwd(af_ctx* c, int B, int H, int W, int Cin, int Cout, int stride, int relu,
                         const void* in, const void* wpack, const float* bias, void* out,
                         float* outf) {
  af_status st = conv_args(c, B, H, W, Cin, Cout, stride);
  if (st != AF_OK) return st;
  if (!in || !wpack || !bias || (!out && !outf)) return fail(c, AF_ERR_ARG, "af_conv3x3_fwd: null pointer");
  AF_KERNEL(AF_K_CONV_FWD,
            af::launch_conv_fwd(c, B, H, W, Cin, Cout, stride, relu, in, wpack, bias, out, outf),
            "conv fwd");
  return AF_OK;
}

af_status af_conv3x3_bwd_data(af_ctx* c, int B, int H, int W, int Cin, int Cout, int stride,
                              const void* dout, const void* wtpack, const void* act, void* din) {
  af_status st = conv_args(c, B, H, W, Cin, Cout, stride);
  if (st != AF_OK) return st;
  if (!dout || !wtpack || !din) return fail(c, AF_ERR_ARG, "af_conv3x3_bwd_data: null pointer");
  AF_KERNEL(AF_K_CONV_BWD_DATA,
            af::launch_conv_bwd_data(c, B, H, W, Cin, Cout, stride, dout, wtpack, act, din),
            "conv bwd data");
  return AF_OK;
}

af_status af_conv3x3_bwd_weight(af_ctx* c, int B, int H, int W, int Cin, int Cout, int stride,
                                const void* in, const void* dout, float* dw, float* db) {
  af_status st = conv_args(c, B, H, W, Cin, Cout, stride);
  if (st != AF_OK) return st;
  if (!in || !dout || !dw || !db) return fail(c, AF_ERR_ARG, "af_conv3x3_bwd_weight: null pointer");
  AF_KERNEL(AF_K_CONV_BWD_WEIGHT,
            af::launch_conv_bwd_weight(c, B, H, W, Cin, Cout, stride, in, dout, dw, db),
            "conv bwd weight");
  return AF_OK;
}

af_status af_conv3x3_bwd_weight_noalloc(af_ctx* c, int B, int H, int W, int Cin, int Cout,
                                        int stride, const void* in, const void* dout, float* dw,
                                        float* db) {
  af_status st = conv_args(c, B, H, W, Cin, Cout, stride);
  if (st != AF_OK) return st;
  if (!in || !dout || !dw || !db)
    return fail(c, AF_ERR_ARG, "af_conv3x3_bwd_weight_noalloc: null pointer");
  if (!c->noalloc_ok)
    return fail(c, AF_ERR_HIP, "af_conv3x3_bwd_weight_noalloc: no address of the scratch array on this device");
  bool too_large = false;
  const hipError_t e = af::launch_conv_bwd_weight_noalloc(c, B, H, W, Cin, Cout, stride, in, dout,
                                                          dw, db, &too_large);
  if (too_large)
    return fail(c, AF_ERR_ARG, "af_conv3x3_bwd_weight_noalloc: partial sums exceed the 29.6 MB scratch array");
  if (e != hipSuccess) return hip_fail(c, e, "conv bwd weight (no allocation)");
  return AF_OK;
}

af_status af_mse_loss(af_ctx* c, int n, const float* out, const float* label, float scale,
                      float* loss_parts, void* dout) {
  if (!c) return AF_ERR_ARG;
  if (n <= 0 || !out || !label || !loss_parts || !dout) return fail(c, AF_ERR_ARG, "af_mse_loss: bad argument");
  AF_HIP(hipSetDevice(c->device), "hipSetDevice");
  AF_HIP(af::launch_mse(c, n, out, label, scale, loss_parts, dout), "mse");
  return AF_OK;
}

af_status af_adam_update(af_ctx* c, int n, const af_adam_params* ap, int step, float* p, float* m,
                         float* v, const float* g) {
  if (!c) return AF_ERR_ARG;
  if (n <= 0 || !ap || step < 1 || !p || !m || !v || !g) return fail(c, AF_ERR_ARG, "af_adam_update: bad argument");
  AF_HIP(hipSetDevice(c->device), "hipSetDevice");
  AF_HIP(af::launch_adam_vec(c, n, ap, step, p, m, v, g), "adam");
  return AF_OK;
}

af_status af_features(af_ctx* c, long long n, int C, const float* maps, const float* shift,
                      const float* scale, void* out) {
  if (!c) return AF_ERR_ARG;
  if (n <= 0 || C <= 0 || !maps || !shift || !scale || !out) return fail(c, AF_ERR_ARG, "af_features: bad argument");
  AF_HIP(hipSetDevice(c->device), "hipSetDevice");
  AF_HIP(af::launch_features(c, n, C, maps, shift, scale, out), "features");
  return AF_OK;
}

af_status af_polar_to_grid(af_ctx* c, const float* map, int nr, int nt, double r0, double dr,
                           double t0, double dt, int nx, int nz, double x0, double z0, double dx,
                           double dz, float s_base, float scale, float s_lo, float s_hi,
                           float* s) {
  if (!c) return AF_ERR_ARG;
  if (!map || !s || nr < 2 || nt < 2 || nx < 1 || nz < 1 || !(dr > 0) || !(dt > 0) ||
      !(dx > 0) || !(dz > 0))
    return fail(c, AF_ERR_ARG, "af_polar_to_grid: bad argument");
  if (!(s_lo > 0.f) || !(s_hi >= s_lo) || !std::isfinite(s_hi))
    return fail(c, AF_ERR_ARG, "af_polar_to_grid: need 0 < s_lo <= s_hi");
  AF_HIP(hipSetDevice(c->device), "hipSetDevice");
  AF_HIP(af::launch_polar_to_grid(c, map, nr, nt, r0, dr, t0, dt, nx, nz, x0, z0, dx, dz, s_base,
                                  scale, s_lo, s_hi, s),
         "polar_to_grid");
  return AF_OK;
}

af_status af_set_profiling(af_ctx* c, int enable) {
  if (!c) return AF_ERR_ARG;
  c->prof_on = enable != 0;
  return AF_OK;
}

af_status af_profile_read(af_ctx* c, double* ms, long long* calls) {
  if (!c || !ms || !calls) return AF_ERR_ARG;
  for (int k = 0; k < AF_K_COUNT; ++k) {
    ms[k] = 0.0;
    calls[k] = 0;
  }
  AF_HIP(c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize(), "profile sync");
  for (auto& pe : c->ev_pending) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, pe.second.first, pe.second.second) == hipSuccess) {
      ms[pe.first] += t;
      calls[pe.first] += 1;
    }
    c->ev_pool.push_back(pe.second.first);
    c->ev_pool.push_back(pe.second.second);
  }
  c->ev_pending.clear();
  return AF_OK;
}

af_status af_query(af_ctx* c, int what, long long* out) {
  if (!c || !out) return AF_ERR_ARG;
  if (!c->has_geom) return fail(c, AF_ERR_STATE, "af_query: no geometry");
  switch (what) {
    case AF_Q_P: *out = c->P; break;
    case AF_Q_P_INTERNAL: *out = c->P_int; break;
    case AF_Q_NBLK: *out = c->nb; break;
    case AF_Q_GBLK_ELEMS: *out = (long long)c->nb * c->nb * c->P_int; break;
    case AF_Q_ACTIVE_PAIRS: *out = c->active_pairs; break;
    case AF_Q_ACTIVE_SAMPLES: *out = c->active_samples; break;
    case AF_Q_TILES: *out = c->n_tiles; break;
    case AF_Q_NA_MAX: *out = c->na_max; break;
    case AF_Q_NBA_MAX: *out = c->nba_max; break;
    case AF_Q_WIDE_TILES: *out = c->n_wide; break;
    case AF_Q_CHUNKS: *out = (long long)c->chunks.size(); break;
    case AF_Q_DEVICE_BYTES: {
      long long b = 0;
      for (const af::DBuf* d :
           {&c->d_elem, &c->d_ptpol, &c->d_ptxy, &c->d_prange, &c->d_tiles, &c->d_tabwork,
            &c->d_daswork, &c->d_order, &c->d_i2c, &c->d_c2i, &c->d_cnn_part, &c->d_ray_uv,
            &c->d_ray_l2, &c->d_chan, &c->d_s, &c->d_gdev, &c->d_regg, &c->d_scal, &c->d_tab,
            &c->d_bblk, &c->d_gT, &c->d_gsb, &c->d_part, &c->d_gpad, &c->d_gpart, &c->d_gsum,
            &c->d_grad, &c->d_terms, &c->d_maps, &c->d_gtp, &c->d_tbase, &c->d_wide,
            &c->d_cmpe_wide, &c->d_dyn_base, &c->d_elemf, &c->d_tstat})
        b += (long long)d->bytes;
      *out = b;
      break;
    }
    default: return fail(c, AF_ERR_ARG, "af_query: unknown item");
  }
  return AF_OK;
}

}  // extern "C"
