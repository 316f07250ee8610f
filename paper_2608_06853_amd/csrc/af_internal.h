// Internal declarations of the library: context, device buffers and the launch
// wrappers of every kernel (one translation unit per kernel family).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/af.h"
#include "af_device.h"

namespace af {

// Growable device buffer owned by a context.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  hipError_t ensure(size_t n) {
    if (n <= bytes) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Static geometry passed by value to kernels.
struct Geo {
  int n_elem, ns, block, nblk, nsub, n_seg, patch2, pps;
  long long P;            // internal points (multiple of TILE)
  double fs, fd, t0, t_ttp;
  double dlens, icl;      // lens thickness, 1/c_lens
  int nsearch;            // discrete refraction candidates (0: continuous root)
  int flat;               // linear array with a flat lens (else the concentric arc)
  // slowness grid
  int nx, nz, W;          // W = nx + 3 (padded row stride)
  float x0, z0, idx, idz;
};

struct TableArgs {
  Geo g;
  const double4* elem;    // (R, sin, cos, 0) polar geometry of each element
  const double4* ptpol;   // (rho, sin, cos, 0) polar geometry of each point
  const float2* ptxy;     // point (x, z)
  const int2* prange;     // active element range [lo, hi] of each point
  const int4* tiles;      // (LO, HI, bLO, bHI)
  const int2* work;       // (tile, first element of a chunk of TAB_CHUNK)
  int n_work;             // work items
  const float* gdev;      // padded deviation grid s - s_med
  const double* scal;     // scal[0] = c_med, scal[1] = s_med
  TabEntry* tab;          // [n_elem][P]
  float2* ray_uv;         // [n_elem][P] ray start (refraction point) in grid coordinates
  float* ray_l2;          // [n_elem][P] medium leg length
};
constexpr int TAB_CHUNK = 8;

struct DasArgs {
  Geo g;
  const TabEntry* tab;
  const float2* iq;       // [N][N][ns]
  const int4* tiles;
  const int2* prange;     // active element range of every point
  const int2* work;       // (tile, rx block) for the forward
  const int* order;       // tile order for the adjoint
  float2* bblk;           // [nb][nb][P]  (forward output)
  const float2* gblk;     // [nb][nb][P]  (adjoint input)
  const double* gscal;    // null: gblk is final; else dL/dB = gblk * gscal[5] + gsb[p]
  const float2* gsb;      // [P] speckle-brightness gradient per point
  float* gT;              // [n_elem][P]  dL/dT, receive role (adjoint output)
  float* gT2;             // [n_elem][P]  dL/dT, transmit role (atomic adds; default mode)
  float* gtp;             // deterministic mode: transmit-role partial sums, one slab per
                          // (tile, receive block)
  const long long* tbase; // [n_tiles] offset of a tile's slabs in gtp
};

struct CmpeArgs {
  Geo g;
  const int4* tiles;
  const float2* bblk;     // input block images
  float2* gout;           // output: unscaled dL_sum/dB^blk (may alias bblk)
  float2* gsb;            // [P] speckle-brightness gradient per centre point
  double* part;           // [n_sub_tiles][4] (sum err, n_valid, sum |B|^2, 0)
  float* map_cmpe;        // [P/patch2 internal pixel slots] or null
  float* map_cf;          // same, or null
  float* map_cmcc;        // same, or null
  float2* img;            // [P] full image or null
  float rho_thresh;
  float sb_scale;         // -2 w_sb / (sb_ref n_pix)
  int write_g;
  // Tiles whose span of active blocks is too wide for LDS keep their subaperture
  // images and pair entries in device memory instead: wide[tile] is the tile's
  // index among them (-1: the LDS path), each of its 4 sub-tiles owns wstride
  // float2 of wscr.
  const int* wide;
  float2* wscr;
  long long wstride;
  // The LDS path runs in one or two launches by the dynamic LDS a tile needs (in
  // float2): a launch takes the tiles with need in (need_lo, need_hi].
  long long need_lo, need_hi;
};

// Per-tile result of the dynamic-grid point update: active element range, whether
// some point's active elements are not contiguous, active rays and samples.
struct TileStat {
  int lo, hi, bad, pad;
  long long pairs, samples;
};

struct PathArgs {
  Geo g;
  const float2* ray_uv;   // ray start and medium leg of every table entry (k_table)
  const float* ray_l2;
  const float2* ptxy;
  const int2* prange;
  const int4* tiles;
  const int* order;
  const float* gT;        // dL/dT [n_elem][P], receive role
  const float* gT2;       // dL/dT [n_elem][P], transmit role (default mode)
  const float* gtp;       // deterministic mode: transmit-role slabs (DasArgs::gtp)
  const long long* tbase;
  float* gpart;           // [n_wg][padded nodes] per-workgroup partial grids
};

// The tiles the hot-path kernels of one launch cover: all of them, or one chunk
// of consecutive tiles in bounded-memory mode (af_set_memory_budget).  Per-tile
// and per-point arrays are offset to the chunk's first tile, so a kernel sees the
// chunk as a whole problem of n_tiles tiles and P points; the [n_elem][P] and
// [nb][nb][P] buffers hold one chunk at a time, with stride P.
struct View {
  int t0 = 0, n_tiles = 0;    // first tile, tiles
  long long p0 = 0, P = 0;    // first internal point, points (n_tiles * TILE)
  const int4* tiles = nullptr;
  const int2* prange = nullptr;
  const float2* ptxy = nullptr;
  const double4* ptpol = nullptr;
  const int2* tabwork = nullptr;  // work lists with chunk-local tile indices
  int n_tab_work = 0;
  const int2* daswork = nullptr;
  int n_das_work = 0;
  const int* order = nullptr;
  int n_order = 0;
  const int* wide = nullptr;      // chunk-local index among the chunk's wide tiles
  int n_wide = 0;
  const long long* tbase = nullptr;  // chunk-local slab offsets (deterministic mode)
  float* map_cmpe = nullptr;      // the chunk's per-pixel slots of the three maps
  float* map_cf = nullptr;
  float* map_cmcc = nullptr;
  double* part = nullptr;         // the chunk's sub-tile partial sums
  float2* gsb = nullptr;          // the chunk's points
};

// Work lists and scratch needs of one chunk (offsets into the concatenated lists).
struct Chunk {
  int t0 = 0, n_tiles = 0;
  int tab_off = 0, n_tab = 0, das_off = 0, n_das = 0, ord_off = 0, n_ord = 0;
  int n_wide = 0;
  long long n_gtp = 0;
};

}  // namespace af

struct af_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool noalloc_ok = false;  // the device's no-allocation scratch address is known
  std::string err;
  bool has_geom = false, has_lens = false, has_grid = false;

  // geometry (host, caller order)
  int N = 0, n_pix = 0, patch = 3, M = 9, Ns = 0, S = 1, nb = 0, nsub = 0, n_seg = 0;
  double spacing = 0, fs = 0, t0 = 0, fd = 0, fnum = 0;
  std::vector<double> elem_xz, pts_xz;      // [N][2], [P][2] caller order
  std::vector<double> elem_R, elem_pol;     // radius, polar angle
  // internal layout
  int pps = 0, ppt = 0, n_tiles = 0;
  long long P = 0, P_int = 0;
  std::vector<int> i2c;                     // internal point -> caller point (-1 pad)
  std::vector<int> h_lo, h_hi;              // host staging of the geometry set-up
  std::vector<double4> h_ptpol;
  std::vector<float2> h_ptxy;
  std::vector<int2> h_prange;
  std::vector<int> c2i;                     // caller point -> internal point
  std::vector<int> prange_lo, prange_hi;    // per internal point
  std::vector<int> tile_lo, tile_hi;
  int na_max = 0, nba_max = 0;
  long long need_lds = 0;  // largest dynamic LDS (float2) of a tile on the CMPE stage's LDS path
  int n_wide = 0;      // tiles on its device-memory path
  long long wstride = 0;
  long long active_pairs = 0, active_samples = 0;
  std::vector<double4> elem_frame;          // element (x, z, cos, sin) of the orientation of Eq. 3
  std::vector<double> pix_xz;               // caller pixel centres of af_set_geometry [n_pix][2]
  // dynamic CMPE grid (af_set_dynamic_grid): the pixels of af_set_geometry are the
  // layout of speed dyn_cref; af_set_sweep_speed moves them on the device
  bool dyn_on = false;
  double dyn_cref = 1.54, dyn_fc = 1.0, dyn_cmin = 1.54, dyn_cmax = 1.54, dyn_c = 1.54;
  double dyn_box[4] = {0, 0, 0, 0};         // x_lo, x_hi, z_lo, z_hi of every point at every speed
  double dyn_ang[2] = {0, 0};               // polar angle (x on a line) range of the same
  af::DBuf d_dyn_base, d_elemf, d_tstat;
  // chunks of consecutive tiles (one chunk holding every tile unless a memory
  // budget is set), their work lists, and the view of the current launch
  size_t mem_budget = 0;                    // bytes for the chunk-sized buffers; 0: none
  std::vector<af::Chunk> chunks;
  long long P_chunk = 0;                    // points of the largest chunk
  int wide_max = 0;                         // most wide tiles of a chunk
  long long gtp_max = 0;                    // most slab floats of a chunk
  af::View v;
  void select(int k);                       // v := chunk k
  bool bounded() const { return chunks.size() > 1; }

  // lens: the physical lens (d_lens_phys, c_lens, t_ttp_phys) and the beamformer's
  // model of it -- the lens thickness its rays refract through (d_lens: 0 for the
  // straight-ray models) and the scalar added to every round trip (t_ttp)
  int lens_mode = AF_LENS_BENT;
  double d_lens_phys = 0, t_ttp_phys = 0, c_ref = 1.54;
  double d_lens = 0, c_lens = 1, t_ttp = 0;
  int n_search = 0;
  bool flat = false;      // linear array: every element on one line z = const
  // grid
  int nx = 0, nz = 0;
  double x0 = 0, z0 = 0, dx = 1, dz = 1;
  float rho_last = 0.9f;

  // device buffers
  af::DBuf d_elem, d_ptpol, d_ptxy, d_prange, d_tiles, d_tabwork, d_daswork, d_order, d_i2c,
      d_c2i;
  af::DBuf d_cnn_part;
  af::DBuf d_ray_uv, d_ray_l2;  // per table entry: ray start (grid coordinates), medium leg
  af::DBuf d_chan;  // receive-channel images, allocated by the coherence calls only
  // d_tab, d_ray_uv, d_ray_l2, d_bblk, d_gT: one chunk ([.][P_chunk]); d_gsum: one
  // grid of path-adjoint sums per chunk
  af::DBuf d_s, d_gdev, d_regg, d_scal, d_tab, d_bblk, d_gT, d_gsb, d_part, d_gpad, d_gpart,
      d_gsum, d_grad, d_terms, d_maps;
  // Transmit-role sums of dL/dT: for every tile and receive block jb of its range
  // one slab [element e - LO][TILE] of sums over the receive elements of jb; the
  // slabs of a tile follow in jb order from d_tbase[tile].
  af::DBuf d_gtp, d_tbase;
  af::DBuf d_wide, d_cmpe_wide;  // CMPE stage of wide tiles (CmpeArgs::wide, wscr)
  bool det = false;  // deterministic mode (af_set_deterministic)

  af::Geo geo() const;

  // kernel timing (af_set_profiling)
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  hipEvent_t ev_get() {
    hipEvent_t e = nullptr;
    if (!ev_pool.empty()) {
      e = ev_pool.back();
      ev_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  ~af_ctx() {
    for (auto& p : ev_pending) {
      (void)hipEventDestroy(p.second.first);
      (void)hipEventDestroy(p.second.second);
    }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
  }
};

namespace af {
// launch wrappers (return hipGetLastError())
hipError_t launch_prepare_grid(af_ctx* c, const float* s, int nx, int nz, float* gdev, double* scal,
                               int do_reg, const af_loss_params* lp, float* regg);
hipError_t launch_table(af_ctx* c);
hipError_t launch_das_fwd(af_ctx* c, const float2* iq, float2* bblk);
// Dynamic LDS (float2) of the CMPE stage for a tile spanning blocks bLO..bHI (its
// pair range clamped at the array's ends), and whether it fits one workgroup's LDS
long long cmpe_need(int bLO, int bHI, int nsub, int pps);
bool cmpe_fits_lds(int bLO, int bHI, int nsub, int pps);
long long cmpe_wide_stride(int nba, int pps);  // float2 per sub-tile of a wide tile
hipError_t launch_cmpe(af_ctx* c, const float2* bblk, float2* gout, int write_g, float rho,
                       float sb_scale, float* map_cmpe, float* map_cf, float* map_cmcc,
                       float2* img);
hipError_t launch_finalize(af_ctx* c, const af_loss_params* lp, float* terms);
hipError_t launch_gscale(af_ctx* c, float2* gblk);
// scaled = false: gblk still lacks its final scale, which the adjoint applies
hipError_t launch_das_adj(af_ctx* c, const float2* iq, const float2* gblk, bool scaled);
// receive-channel images X[N][P_int] (internal order), their caller-order export,
// and the per-pixel lag-one coherence from them
hipError_t launch_channel_images(af_ctx* c, const float2* iq, float2* X);
hipError_t launch_export_rx(af_ctx* c, const float2* X, float2* out);
hipError_t launch_loc(af_ctx* c, const float2* X, float* loc);
hipError_t launch_path_adj(af_ctx* c, float* out);  // the view's grid sums -> out [nodes]
hipError_t launch_sum_grids(af_ctx* c, float* parts, int n, float* out);  // parts is overwritten
// dynamic grid: points at k = c_g / c_ref with patch spacing `spacing` from the lens
// surface rl, their active element ranges, and per tile the statistics in tstat
hipError_t launch_sweep_points(af_ctx* c, double k, double spacing, double rl, TileStat* tstat);
hipError_t launch_fill(af_ctx* c, float* x, int n, float v);
hipError_t launch_grad_fold(af_ctx* c, float* grad);
hipError_t launch_adam(af_ctx* c, const af_adam_params* ap, int step, float* s, float* m,
                       float* v, const float* grad);
hipError_t launch_export_T(af_ctx* c, float* out);
hipError_t launch_export_images(af_ctx* c, const float2* bblk, float2* blk_out, float2* img_out,
                                float* maps_out);
hipError_t launch_simulate(af_ctx* c, int n_scat, const double* scat_xz, const float* amp,
                           int nx, int nz, double x0, double z0, double dx, double dz,
                           const float* s_true, int n_seg, double fc, double frac_bw,
                           float2* iq);
hipError_t launch_conv_fwd(af_ctx* c, int B, int H, int W, int Cin, int Cout, int stride, int relu,
                           const void* in, const void* wp, const float* bias, void* out,
                           float* outf);
hipError_t launch_conv_bwd_data(af_ctx* c, int B, int H, int W, int Cin, int Cout, int stride,
                                const void* dout, const void* wtp, const void* act, void* din);
hipError_t launch_conv_bwd_weight(af_ctx* c, int B, int H, int W, int Cin, int Cout, int stride,
                                  const void* in, const void* dout, float* dw, float* db);
// The same with its partial sums in the library's static device array: no
// allocation.  noalloc_scratch_init takes the array's address on `device` (which
// must be current) once; *too_large reports a shape beyond the array.
hipError_t noalloc_scratch_init(int device);
hipError_t launch_conv_bwd_weight_noalloc(af_ctx* c, int B, int H, int W, int Cin, int Cout,
                                          int stride, const void* in, const void* dout, float* dw,
                                          float* db, bool* too_large);
hipError_t launch_conv_pack(af_ctx* c, int Cin, int Cout, const float* w, void* wp, void* wtp);
hipError_t launch_mse(af_ctx* c, int n, const float* out, const float* label, float scale,
                      float* loss_parts, void* dout);
hipError_t launch_adam_vec(af_ctx* c, int n, const af_adam_params* ap, int step, float* p, float* m,
                           float* v, const float* g);
hipError_t launch_features(af_ctx* c, long long n, int C, const float* maps, const float* shift,
                           const float* scale, void* out);
hipError_t launch_polar_to_grid(af_ctx* c, const float* map, int nr, int nt, double r0, double dr,
                                double t0, double dt, int nx, int nz, double x0, double z0,
                                double dx, double dz, float s_base, float scale, float s_lo,
                                float s_hi, float* s);
}  // namespace af
