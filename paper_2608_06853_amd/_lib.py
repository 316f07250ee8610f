"""ctypes binding of libaf.so (include/af.h).  Argument marshalling only.

Device buffers are torch CUDA tensors (torch supplies memory and the stream);
host arrays are NumPy float64.  Every method maps one-to-one onto an ``af_*``
entry point and raises ``AfError`` on a non-zero status.  There is no fallback:
if the library is not built, importing this module fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2608_06853_amd.build` "
                      "(or __graft_entry__.build()); there is no CPU fallback")

# torch first: its HIP runtime is then the one libaf.so binds to (both carry the
# soname libamdhip64.so.7).  Loaded the other way round, torch brings a second HIP
# runtime into the process and the library's runtime finds no usable device.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

AF_OK, AF_ERR_ARG, AF_ERR_STATE, AF_ERR_HIP, AF_ERR_OOM, AF_ERR_NUMERIC = 0, -1, -2, -3, -4, -5
TERM_CMPE, TERM_TV, TERM_SV, TERM_SB, TERM_TOTAL, TERM_NVALID, TERM_CMED = range(7)
N_TERMS = 8
LENS_BENT, LENS_CONVENTIONAL, LENS_NONE = 0, 1, 2
LENS_MODES = {"bent": LENS_BENT, "conventional": LENS_CONVENTIONAL, "none": LENS_NONE}
(Q_P, Q_P_INTERNAL, Q_NBLK, Q_GBLK_ELEMS, Q_ACTIVE_PAIRS, Q_ACTIVE_SAMPLES, Q_TILES, Q_NA_MAX,
 Q_NBA_MAX, Q_WIDE_TILES, Q_CHUNKS, Q_DEVICE_BYTES) = range(12)

EXPORTS = [
    "af_create", "af_destroy", "af_last_error", "af_set_geometry", "af_set_lens",
    "af_set_refraction_search", "af_set_deterministic", "af_set_memory_budget", "af_set_slowness", "af_beamform", "af_loss_and_grad", "af_forward", "af_backward",
    "af_autofocus_step", "af_travel_times", "af_set_dynamic_grid", "af_set_sweep_speed",
    "af_sweep", "af_simulate", "af_query", "af_set_profiling",
    "af_profile_read", "af_conv3x3_pack", "af_conv3x3_fwd", "af_conv3x3_bwd_data",
    "af_conv3x3_bwd_weight", "af_conv3x3_bwd_weight_noalloc", "af_mse_loss", "af_adam_update",
    "af_features", "af_polar_to_grid",
]
KERNELS = ["prepare_grid", "table", "das_fwd", "cmpe", "finalize", "gscale", "das_adj",
           "path_adj", "grad_fold", "adam", "export", "conv_fwd", "conv_bwd_data",
           "conv_bwd_weight"]


class LossParams(C.Structure):
    _fields_ = [(n, C.c_float) for n in
                ("w1", "kx1", "kz1", "w2", "kx2", "kz2", "rho_thresh", "w_sb", "sb_ref")]


class AdamParams(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("lr", "beta1", "beta2", "eps")]


_vp = C.c_void_p
_d = C.c_double
_i = C.c_int
_sig = {
    "af_create": (C.c_int, [C.POINTER(_vp), _i, _vp]),
    "af_destroy": (None, [_vp]),
    "af_last_error": (C.c_char_p, [_vp]),
    "af_set_geometry": (C.c_int, [_vp, _i, _vp, _i, _vp, _i, _d, _i, _d, _d, _d, _i, _d, _i]),
    "af_set_lens": (C.c_int, [_vp, _d, _d, _d, _i, _d]),
    "af_set_refraction_search": (C.c_int, [_vp, _i]),
    "af_set_deterministic": (C.c_int, [_vp, _i]),
    "af_set_memory_budget": (C.c_int, [_vp, C.c_size_t]),
    "af_set_slowness": (C.c_int, [_vp, _i, _i, _d, _d, _d, _d, _vp]),
    "af_beamform": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "af_channel_images": (C.c_int, [_vp, _vp, _vp]),
    "af_lag_one_coherence": (C.c_int, [_vp, _vp, _vp]),
    "af_loss_and_grad": (C.c_int, [_vp, _vp, C.POINTER(LossParams), _vp, _vp]),
    "af_forward": (C.c_int, [_vp, _vp, C.POINTER(LossParams), _vp, _vp]),
    "af_backward": (C.c_int, [_vp, _vp, C.POINTER(LossParams), _vp, _vp]),
    "af_autofocus_step": (C.c_int, [_vp, _vp, C.POINTER(LossParams), C.POINTER(AdamParams), _i,
                                    _vp, _vp, _vp, _vp]),
    "af_travel_times": (C.c_int, [_vp, _vp]),
    "af_set_dynamic_grid": (C.c_int, [_vp, _d, _d, _d, _d]),
    "af_set_sweep_speed": (C.c_int, [_vp, _d]),
    "af_sweep": (C.c_int, [_vp, _vp, C.POINTER(LossParams), _i, _vp, _i, _d, _vp,
                           C.POINTER(C.c_double)]),
    "af_simulate": (C.c_int, [_vp, _i, _vp, _vp, _i, _i, _d, _d, _d, _d, _vp, _i, _d, _d, _vp]),
    "af_query": (C.c_int, [_vp, _i, C.POINTER(C.c_longlong)]),
    "af_set_profiling": (C.c_int, [_vp, _i]),
    "af_profile_read": (C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]),
    "af_conv3x3_pack": (C.c_int, [_vp, _i, _i, _vp, _vp, _vp]),
    "af_conv3x3_fwd": (C.c_int, [_vp, _i, _i, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp]),
    "af_conv3x3_bwd_data": (C.c_int, [_vp, _i, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp]),
    "af_conv3x3_bwd_weight": (C.c_int, [_vp, _i, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp]),
    "af_conv3x3_bwd_weight_noalloc": (C.c_int, [_vp, _i, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp]),
    "af_mse_loss": (C.c_int, [_vp, _i, _vp, _vp, C.c_float, _vp, _vp]),
    "af_adam_update": (C.c_int, [_vp, _i, C.POINTER(AdamParams), _i, _vp, _vp, _vp, _vp]),
    "af_features": (C.c_int, [_vp, C.c_longlong, _i, _vp, _vp, _vp, _vp]),
    "af_polar_to_grid": (C.c_int, [_vp, _vp, _i, _i, _d, _d, _d, _d, _i, _i, _d, _d, _d, _d,
                                   C.c_float, C.c_float, C.c_float, C.c_float, _vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class AfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"af status {status}: {msg}")
        self.status = status


def _host(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _dev(t, dtype, numel=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor of ``dtype`` (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    return t.data_ptr()


def loss_params(w1=10.0, kx1=0.01, kz1=0.01, w2=100.0, kx2=0.001, kz2=0.001, rho_thresh=0.9,
                w_sb=0.0, sb_ref=1.0) -> LossParams:
    return LossParams(w1, kx1, kz1, w2, kx2, kz2, rho_thresh, w_sb, sb_ref)


def adam_params(lr=0.003, beta1=0.9, beta2=0.999, eps=1e-8) -> AdamParams:
    return AdamParams(lr, beta1, beta2, eps)


class Context:
    """One af_ctx bound to a device and a torch stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.device = device
        h = _vp()
        st = _lib.af_create(C.byref(h), device, _vp(stream.cuda_stream))
        if st != AF_OK:
            raise AfError(st, _lib.af_last_error(None).decode())
        self._h = h
        self.n_elem = self.n_samples = self.n_pix = self.patch = 0
        self.nx = self.nz = 0

    def close(self):
        if getattr(self, "_h", None):
            _lib.af_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        if st != AF_OK:
            raise AfError(st, _lib.af_last_error(self._h).decode())

    # --- af_set_* -----------------------------------------------------------------
    def set_geometry(self, elem_xz, pix_xz, patch, patch_spacing, n_samples, fs, t0, fd, block,
                     fnum, n_seg):
        e = _host(elem_xz)
        p = _host(pix_xz)
        self.n_elem, self.n_pix = e.size // 2, p.size // 2
        self.patch, self.n_samples = int(patch), int(n_samples)
        self._chk(_lib.af_set_geometry(self._h, self.n_elem, e.ctypes.data, self.n_pix,
                                       p.ctypes.data, int(patch), float(patch_spacing),
                                       int(n_samples), float(fs), float(t0), float(fd), int(block),
                                       float(fnum), int(n_seg)))

    def set_lens(self, d_lens, c_lens, t_ttp=0.0, mode=LENS_BENT, c_ref=1.540):
        self._chk(_lib.af_set_lens(self._h, float(d_lens), float(c_lens), float(t_ttp), int(mode),
                                   float(c_ref)))

    def set_refraction_search(self, n_search: int):
        self._chk(_lib.af_set_refraction_search(self._h, int(n_search)))

    def set_deterministic(self, on: bool):
        self._chk(_lib.af_set_deterministic(self._h, 1 if on else 0))

    def set_memory_budget(self, nbytes: int):
        self._chk(_lib.af_set_memory_budget(self._h, int(nbytes)))

    def set_slowness(self, nx, nz, x0, z0, dx, dz, s):
        import torch
        self.nx, self.nz = int(nx), int(nz)
        self._chk(_lib.af_set_slowness(self._h, int(nx), int(nz), float(x0), float(z0), float(dx),
                                       float(dz), _dev(s, torch.float32, nx * nz, "s")))

    # --- hot path -------------------------------------------------------------------
    def _iq(self, iq):
        import torch
        return _dev(iq, torch.complex64, self.n_elem * self.n_elem * self.n_samples, "iq")

    def beamform(self, iq, blk=None, img=None, maps=None):
        import torch
        P = self.n_pix * self.patch ** 2
        nb = self.query(Q_NBLK)
        self._chk(_lib.af_beamform(self._h, self._iq(iq),
                                   _dev(blk, torch.complex64, nb * nb * P, "blk"),
                                   _dev(img, torch.complex64, P, "img"),
                                   _dev(maps, torch.float32, 3 * self.n_pix, "maps")))

    def channel_images(self, iq, out):
        import torch
        P = self.n_pix * self.patch ** 2
        self._chk(_lib.af_channel_images(self._h, self._iq(iq),
                                         _dev(out, torch.complex64, self.n_elem * P, "out")))

    def lag_one_coherence(self, iq, out):
        import torch
        self._chk(_lib.af_lag_one_coherence(self._h, self._iq(iq),
                                            _dev(out, torch.float32, self.n_pix, "out")))

    def loss_and_grad(self, iq, lp: LossParams, terms, grad=None):
        import torch
        self._chk(_lib.af_loss_and_grad(self._h, self._iq(iq), C.byref(lp),
                                        _dev(terms, torch.float32, N_TERMS, "terms"),
                                        _dev(grad, torch.float32, self.nx * self.nz, "grad")))

    def forward(self, iq, lp: LossParams, terms, gblk):
        import torch
        self._chk(_lib.af_forward(self._h, self._iq(iq), C.byref(lp),
                                  _dev(terms, torch.float32, N_TERMS, "terms"),
                                  _dev(gblk, torch.complex64, self.query(Q_GBLK_ELEMS), "gblk")))

    def backward(self, iq, lp: LossParams, gblk, grad):
        import torch
        self._chk(_lib.af_backward(self._h, self._iq(iq), C.byref(lp),
                                   _dev(gblk, torch.complex64, self.query(Q_GBLK_ELEMS), "gblk"),
                                   _dev(grad, torch.float32, self.nx * self.nz, "grad")))

    def autofocus_step(self, iq, lp: LossParams, ap: AdamParams, step, s, m, v, terms):
        import torch
        n = self.nx * self.nz
        self._chk(_lib.af_autofocus_step(self._h, self._iq(iq), C.byref(lp), C.byref(ap), int(step),
                                         _dev(s, torch.float32, n, "s"),
                                         _dev(m, torch.float32, n, "m"),
                                         _dev(v, torch.float32, n, "v"),
                                         _dev(terms, torch.float32, N_TERMS, "terms")))

    def set_dynamic_grid(self, c_ref, fc, c_min, c_max):
        self._chk(_lib.af_set_dynamic_grid(self._h, float(c_ref), float(fc), float(c_min),
                                           float(c_max)))

    def set_sweep_speed(self, c_g):
        self._chk(_lib.af_set_sweep_speed(self._h, float(c_g)))

    def sweep(self, iq, lp, speeds, dynamic, static_c, cmpe_out) -> float:
        """Returns the best speed; cmpe_out (device, float32 [len(speeds)]) gets the CMPE
        of every speed."""
        import torch
        sp = _host(speeds)
        best = C.c_double(0.0)
        self._chk(_lib.af_sweep(self._h, _dev(iq, torch.complex64, None, "iq"), C.byref(lp),
                                sp.size, sp.ctypes.data, int(bool(dynamic)), float(static_c),
                                _dev(cmpe_out, torch.float32, sp.size, "cmpe_out"),
                                C.byref(best)))
        return best.value

    def travel_times(self, out):
        import torch
        P = self.n_pix * self.patch ** 2
        self._chk(_lib.af_travel_times(self._h, _dev(out, torch.float32, self.n_elem * P, "out")))

    def simulate(self, scat_xz, amp, nx, nz, x0, z0, dx, dz, s_true, n_seg, fc, frac_bw, iq):
        import torch
        sx = _host(scat_xz)
        am = np.ascontiguousarray(amp, dtype=np.float32)
        self._chk(_lib.af_simulate(self._h, am.size, sx.ctypes.data, am.ctypes.data, int(nx),
                                   int(nz), float(x0), float(z0), float(dx), float(dz),
                                   _dev(s_true, torch.float32, nx * nz, "s_true"), int(n_seg),
                                   float(fc), float(frac_bw), self._iq(iq)))

    def set_profiling(self, enable: bool):
        self._chk(_lib.af_set_profiling(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{kernel: (total ms, launches)} since the last read (waits for the stream)."""
        n = len(KERNELS)
        ms = (C.c_double * n)()
        calls = (C.c_longlong * n)()
        self._chk(_lib.af_profile_read(self._h, ms, calls))
        return {k: (ms[i], calls[i]) for i, k in enumerate(KERNELS) if calls[i] > 0}

    # --- learned warm start (BF16 tensors are torch.bfloat16) -------------------------
    @staticmethod
    def conv_shapes(Cin, Cout):
        kp = (9 * Cin + 15) // 16 * 16
        ktp = (9 * Cout + 15) // 16 * 16
        return kp, ktp

    def conv3x3_pack(self, Cin, Cout, w, wpack, wtpack=None):
        import torch
        kp, ktp = self.conv_shapes(Cin, Cout)
        self._chk(_lib.af_conv3x3_pack(self._h, Cin, Cout, _dev(w, torch.float32, Cout * 9 * Cin, "w"),
                                       _dev(wpack, torch.bfloat16, 32 * kp, "wpack"),
                                       _dev(wtpack, torch.bfloat16, 32 * ktp, "wtpack")))

    def conv3x3_fwd(self, B, H, W, Cin, Cout, stride, relu, x, wpack, bias, out=None, outf=None):
        import torch
        ho, wo = (H - 1) // stride + 1, (W - 1) // stride + 1
        kp, _ = self.conv_shapes(Cin, Cout)
        self._chk(_lib.af_conv3x3_fwd(self._h, B, H, W, Cin, Cout, stride, int(relu),
                                      _dev(x, torch.bfloat16, B * H * W * Cin, "x"),
                                      _dev(wpack, torch.bfloat16, 32 * kp, "wpack"),
                                      _dev(bias, torch.float32, Cout, "bias"),
                                      _dev(out, torch.bfloat16, B * ho * wo * Cout, "out"),
                                      _dev(outf, torch.float32, B * ho * wo * Cout, "outf")))

    def conv3x3_bwd_data(self, B, H, W, Cin, Cout, stride, dout, wtpack, act, din):
        import torch
        ho, wo = (H - 1) // stride + 1, (W - 1) // stride + 1
        _, ktp = self.conv_shapes(Cin, Cout)
        self._chk(_lib.af_conv3x3_bwd_data(self._h, B, H, W, Cin, Cout, stride,
                                           _dev(dout, torch.bfloat16, B * ho * wo * Cout, "dout"),
                                           _dev(wtpack, torch.bfloat16, 32 * ktp, "wtpack"),
                                           _dev(act, torch.bfloat16, B * H * W * Cin, "act"),
                                           _dev(din, torch.bfloat16, B * H * W * Cin, "din")))

    def conv3x3_bwd_weight(self, B, H, W, Cin, Cout, stride, x, dout, dw, db, noalloc=False):
        """noalloc=True calls af_conv3x3_bwd_weight_noalloc (partial sums in the
        library's static device array, no allocation)."""
        import torch
        ho, wo = (H - 1) // stride + 1, (W - 1) // stride + 1
        fn = _lib.af_conv3x3_bwd_weight_noalloc if noalloc else _lib.af_conv3x3_bwd_weight
        self._chk(fn(self._h, B, H, W, Cin, Cout, stride,
                                             _dev(x, torch.bfloat16, B * H * W * Cin, "x"),
                                             _dev(dout, torch.bfloat16, B * ho * wo * Cout, "dout"),
                                             _dev(dw, torch.float32, Cout * 9 * Cin, "dw"),
                                             _dev(db, torch.float32, Cout, "db")))

    def mse_loss(self, out, label, scale, loss_parts, dout):
        import torch
        n = out.numel()
        self._chk(_lib.af_mse_loss(self._h, n, _dev(out, torch.float32, n, "out"),
                                   _dev(label, torch.float32, n, "label"), float(scale),
                                   _dev(loss_parts, torch.float32, (n + 255) // 256, "loss_parts"),
                                   _dev(dout, torch.bfloat16, n, "dout")))

    def adam_update(self, ap: AdamParams, step, p, m, v, g):
        import torch
        n = p.numel()
        self._chk(_lib.af_adam_update(self._h, n, C.byref(ap), int(step),
                                      _dev(p, torch.float32, n, "p"), _dev(m, torch.float32, n, "m"),
                                      _dev(v, torch.float32, n, "v"), _dev(g, torch.float32, n, "g")))

    def features(self, maps, shift, scale, out):
        import torch
        C_ = shift.numel()
        n = maps.numel() // C_
        self._chk(_lib.af_features(self._h, n, C_, _dev(maps, torch.float32, n * C_, "maps"),
                                   _dev(shift, torch.float32, C_, "shift"),
                                   _dev(scale, torch.float32, C_, "scale"),
                                   _dev(out, torch.bfloat16, n * C_, "out")))

    def polar_to_grid(self, pmap, nr, nt, r0, dr, t0, dt, nx, nz, x0, z0, dx, dz, s_base, scale,
                      s_lo, s_hi, s):
        import torch
        self._chk(_lib.af_polar_to_grid(self._h, _dev(pmap, torch.float32, nr * nt, "map"), nr, nt,
                                        float(r0), float(dr), float(t0), float(dt), nx, nz,
                                        float(x0), float(z0), float(dx), float(dz), float(s_base),
                                        float(scale), float(s_lo), float(s_hi),
                                        _dev(s, torch.float32, nx * nz, "s")))

    def query(self, what: int) -> int:
        out = C.c_longlong(0)
        self._chk(_lib.af_query(self._h, int(what), C.byref(out)))
        return int(out.value)
