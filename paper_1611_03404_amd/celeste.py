"""Python binding of libceleste (argument marshalling only).

Every step of the ELBO evaluation and of the trust-region fits runs in the HIP
library; this module only builds the C structs, passes pointers and reads back
results.  It raises if the library is missing: there is no other code path.

Batches are given as structure-of-arrays (one entry per image, CSR offsets per
source).  Pixels given as a NumPy array make a host-memory batch (the library
stages them to the device); a torch tensor on a GPU makes a device-memory batch,
and theta / outputs are then torch tensors on the same device.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libceleste.so")

NP = 27
OK, E_INVALID, E_NOMEM, E_DEVICE, E_UNSUPPORTED = 0, -1, -2, -3, -4
MEM_HOST, MEM_DEVICE = 0, 1
CONVERGED, MAX_ITER, TR_COLLAPSED, NONFINITE, LINE_SEARCH_FAILED = 0, 1, 2, 3, 4
INIT_AS_GIVEN, INIT_PLAIN, INIT_SURROGATE = 0, 1, 2
FLAG_FALLBACK_USED = 1
OPT_CHUNK_PX, OPT_BLOCK, OPT_USE_GRAPH, OPT_PROFILE, OPT_VARIANT = 1, 2, 3, 4, 5
OPT_TILE_W, OPT_VALUE_BLOCK, OPT_VALUE_TILE_W, OPT_EXACT_ZERO, OPT_PERSISTENT, OPT_TR_CHOLESKY = 6, 7, 8, 9, 10, 11
OPT_FP64_SUMS = 12
OPT_TRIAL_DERIVATIVES = 13

IMAGE_DT = np.dtype([
    ("band", "<i4"), ("h", "<i4"), ("w", "<i4"), ("pitch", "<i4"), ("n_psf", "<i4"), ("nbr_pitch", "<i4"),
    ("origin", "<f8", (2,)), ("wcs", "<f8", (6,)), ("sky", "<f8"), ("calib", "<f8"), ("psf", "<f8", (4, 6)),
    ("pixels", "<u8"), ("nbr_mean", "<u8"), ("nbr_var", "<u8"),
])
PRIOR_DT = np.dtype([("p_star", "<f8"), ("r_mean", "<f8", (2,)), ("r_var", "<f8", (2,)),
                     ("c_mean", "<f8", (2, 4)), ("c_cov", "<f8", (2, 4, 4))])
PROF_DT = np.dtype([("n_exp", "<i4"), ("n_dev", "<i4"), ("exp_amp", "<f8", (8,)), ("exp_var", "<f8", (8,)),
                    ("dev_amp", "<f8", (8,)), ("dev_var", "<f8", (8,))])
RESULT_DT = np.dtype([("elbo", "<f8"), ("pred_gain", "<f8"), ("delta", "<f8"), ("iters", "<i4"),
                      ("status", "<i4"), ("n_full_evals", "<i4"), ("flags", "<i4"), ("n_accepted", "<i4"),
                      ("reserved", "<i4")])


class CBatch(ctypes.Structure):
    _fields_ = [("n_sources", ctypes.c_int32), ("mem_kind", ctypes.c_int32), ("image_offsets", ctypes.c_void_p),
                ("images", ctypes.c_void_p), ("prior", ctypes.c_void_p), ("profiles", ctypes.c_void_p)]


class FitOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("init_mode", ctypes.c_int32), ("pred_rtol", ctypes.c_double),
                ("curv_tol", ctypes.c_double), ("delta0", ctypes.c_double), ("delta_max", ctypes.c_double),
                ("delta_min", ctypes.c_double), ("eta", ctypes.c_double), ("u_box", ctypes.c_double),
                ("poll_every", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class LbfgsOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("memory", ctypes.c_int32), ("max_backtracks", ctypes.c_int32),
                ("init_mode", ctypes.c_int32), ("poll_every", ctypes.c_int32), ("max_loops", ctypes.c_int32),
                ("pred_rtol", ctypes.c_double), ("armijo_c1", ctypes.c_double), ("u_box", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("full_px", ctypes.c_int64), ("value_px", ctypes.c_int64), ("full_launches", ctypes.c_int64),
                ("value_launches", ctypes.c_int64), ("iterations", ctypes.c_int64), ("ms_setup", ctypes.c_double),
                ("ms_full", ctypes.c_double), ("ms_reduce_full", ctypes.c_double), ("ms_tr", ctypes.c_double),
                ("ms_value", ctypes.c_double), ("ms_reduce_value", ctypes.c_double), ("ms_accept", ctypes.c_double),
                ("ms_host_pack", ctypes.c_double), ("ms_prepare", ctypes.c_double), ("ms_start", ctypes.c_double),
                ("ms_loop", ctypes.c_double), ("ms_results", ctypes.c_double), ("lr_launches", ctypes.c_int64),
                ("ms_lr", ctypes.c_double), ("grad_px", ctypes.c_int64), ("grad_launches", ctypes.c_int64),
                ("ms_grad", ctypes.c_double), ("ms_reduce_grad", ctypes.c_double), ("ms_lbfgs", ctypes.c_double),
                ("tr_interior", ctypes.c_int64), ("tr_boundary", ctypes.c_int64), ("tr_eigen", ctypes.c_int64),
                ("ms_net", ctypes.c_double), ("tr_sweeps", ctypes.c_int64), ("tr_sweep_cap", ctypes.c_int64),
                ("tr_newton_steps", ctypes.c_int64), ("fit_grid_blocks", ctypes.c_int64),
                ("trial_full_px", ctypes.c_int64), ("taken_px", ctypes.c_int64)]


class TuneResult(ctypes.Structure):
    _fields_ = [("chunk_px", ctypes.c_int32), ("block", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("value_block", ctypes.c_int32), ("value_tile_w", ctypes.c_int32),
                ("n_candidates", ctypes.c_int32), ("from_cache", ctypes.c_int32), ("sample_sources", ctypes.c_int64),
                ("sample_px", ctypes.c_int64), ("full_ms", ctypes.c_double), ("value_ms", ctypes.c_double),
                ("default_full_ms", ctypes.c_double), ("default_value_ms", ctypes.c_double),
                ("vector_full_ms", ctypes.c_double), ("matrix_full_ms", ctypes.c_double)]


class CFields(ctypes.Structure):
    _fields_ = [("n_fields", ctypes.c_int32), ("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("img_field", ctypes.c_void_p), ("mean", ctypes.c_void_p),
                ("var", ctypes.c_void_p)]


class CelesteError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libceleste error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libceleste.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1611_03404_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.celeste_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    lib.celeste_ctx_destroy.argtypes = [vp]
    lib.celeste_ctx_destroy.restype = None
    lib.celeste_last_error.restype = ctypes.c_char_p
    lib.celeste_ctx_set_option.argtypes = [vp, ctypes.c_int, i64]
    lib.celeste_struct_size.argtypes = [ctypes.c_int]
    lib.celeste_struct_size.restype = ctypes.c_size_t
    lib.celeste_fit_opts_default.argtypes = [ctypes.POINTER(FitOpts)]
    lib.celeste_fit_opts_default.restype = None
    lib.celeste_lbfgs_opts_default.argtypes = [ctypes.POINTER(LbfgsOpts)]
    lib.celeste_lbfgs_opts_default.restype = None
    lib.celeste_lbfgs_fit.argtypes = [vp, ctypes.POINTER(CBatch), vp, ctypes.POINTER(LbfgsOpts), vp, vp]
    lib.celeste_batch_fit_sampled.argtypes = [vp, ctypes.POINTER(CBatch), vp, ctypes.POINTER(FitOpts), vp, vp,
                                              ctypes.c_double, ctypes.c_double, vp, vp]
    lib.celeste_elbo_eval.argtypes = [vp, ctypes.POINTER(CBatch), vp, vp, vp, vp, vp]
    lib.celeste_elbo_eval_noalloc.argtypes = [vp, ctypes.POINTER(CBatch), vp, vp, vp, vp, vp]
    lib.celeste_lr_covariance_from_hessian.argtypes = [vp, i64, ctypes.c_int, vp, vp, ctypes.c_double, vp, vp, vp,
                                                       vp, vp]
    lib.celeste_lr_covariance.argtypes = [vp, ctypes.POINTER(CBatch), vp, vp, ctypes.c_double, vp, vp, vp]
    lib.celeste_elbo_eval_sampled.argtypes = [vp, ctypes.POINTER(CBatch), vp, vp, vp, ctypes.c_double, vp, vp, vp,
                                              vp]
    lib.celeste_newton_fit.argtypes = [vp, ctypes.POINTER(CBatch), vp, ctypes.POINTER(FitOpts), vp]
    lib.celeste_batch_fit.argtypes = [vp, ctypes.POINTER(CBatch), vp, ctypes.POINTER(FitOpts), vp, vp]
    lib.celeste_ctx_get_stats.argtypes = [vp, ctypes.POINTER(Stats), ctypes.c_int]
    lib.celeste_net_num_params.restype = i64
    lib.celeste_net_create.argtypes = [vp, vp, i64, vp, vp, ctypes.POINTER(vp)]
    lib.celeste_net_destroy.argtypes = [vp]
    lib.celeste_net_destroy.restype = None
    lib.celeste_net_get_params.argtypes = [vp, vp]
    lib.celeste_net_loss_grad.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp]
    lib.celeste_net_forward.argtypes = [vp, vp, i64, vp]
    lib.celeste_net_train.argtypes = [vp, vp, vp, i64, vp, ctypes.c_int, ctypes.c_int, ctypes.c_float, vp]
    lib.celeste_make_patches.argtypes = [vp, ctypes.POINTER(CBatch), vp, vp]
    lib.celeste_ctx_set_surrogate.argtypes = [vp, vp]
    lib.celeste_theta_to_psi.argtypes = [vp, vp, i64, ctypes.c_double, vp]
    lib.celeste_render_fields.argtypes = [vp, ctypes.POINTER(CBatch), vp, ctypes.POINTER(CFields)]
    lib.celeste_neighbour_arrays.argtypes = [vp, ctypes.POINTER(CBatch), vp, ctypes.POINTER(CFields), vp, vp, vp]
    lib.celeste_start.argtypes = [vp, ctypes.POINTER(CBatch), vp, ctypes.POINTER(FitOpts), vp]
    lib.celeste_psi_to_theta.argtypes = [vp, vp, i64, ctypes.c_double, vp]
    lib.celeste_autotune.argtypes = [vp, ctypes.POINTER(CBatch), vp, i64, ctypes.c_char_p, ctypes.POINTER(TuneResult)]
    lib.celeste_colour_sources.argtypes = [ctypes.POINTER(CBatch), vp, vp]
    lib.celeste_update_fields.argtypes = [vp, ctypes.POINTER(CBatch), vp, vp, ctypes.POINTER(CFields)]
    lib.celeste_field_elbo.argtypes = [vp, ctypes.POINTER(CBatch), vp, ctypes.POINTER(CFields), vp, vp, vp]
    for name in ("celeste_ctx_create", "celeste_ctx_set_option", "celeste_elbo_eval", "celeste_elbo_eval_sampled",
                 "celeste_lr_covariance", "celeste_lr_covariance_from_hessian",
                 "celeste_newton_fit",
                 "celeste_batch_fit", "celeste_ctx_get_stats", "celeste_net_create", "celeste_net_get_params",
                 "celeste_net_loss_grad", "celeste_net_forward", "celeste_net_train", "celeste_make_patches",
                 "celeste_ctx_set_surrogate", "celeste_theta_to_psi", "celeste_psi_to_theta",
                 "celeste_render_fields", "celeste_neighbour_arrays", "celeste_start", "celeste_autotune",
                 "celeste_colour_sources", "celeste_update_fields", "celeste_field_elbo"):
        getattr(lib, name).restype = ctypes.c_int
    sizes = [lib.celeste_struct_size(k) for k in range(9)]
    expect = [IMAGE_DT.itemsize, PRIOR_DT.itemsize, PROF_DT.itemsize, ctypes.sizeof(CBatch),
              ctypes.sizeof(FitOpts), RESULT_DT.itemsize, ctypes.sizeof(Stats), ctypes.sizeof(TuneResult),
              ctypes.sizeof(LbfgsOpts)]
    if sizes != expect:
        raise RuntimeError(f"ABI struct sizes differ: library {sizes}, binding {expect}")
    _lib = lib
    return lib


def _check(code):
    if code != OK:
        raise CelesteError(code, load().celeste_last_error().decode())


def colour_sources(batch: Batch):
    """Conflict-free colours (celeste_colour_sources): returns (colour per source, number of colours)."""
    col = np.zeros(batch.n_sources, dtype=np.int32)
    n = ctypes.c_int32()
    _check(load().celeste_colour_sources(ctypes.byref(batch.c), col.ctypes.data, ctypes.byref(n)))
    return col, n.value


def default_lbfgs_opts(**kw):
    o = LbfgsOpts()
    load().celeste_lbfgs_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_opts(**kw):
    o = FitOpts()
    load().celeste_fit_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x):
    if _is_torch(x):
        return x.data_ptr()
    return x.ctypes.data


class Batch:
    """ABI batch from structure-of-arrays image metadata (keeps its arrays alive)."""

    def __init__(self, src_img_off, band, h, w, pitch, origin, wcs, sky, calib, psf, npsf, pixels, pix_off,
                 prior, profiles, nbr_mean=None, nbr_var=None, nbr_off=None, nbr_pitch=None):
        n_img = int(len(band))
        self.device = _is_torch(pixels) and pixels.is_cuda
        if self.device:
            if pixels.dtype.__repr__() != "torch.float32" or not pixels.is_contiguous():
                raise ValueError("device pixels must be a contiguous float32 tensor")
        else:
            pixels = np.ascontiguousarray(pixels, dtype=np.float32)
        self._keep = [pixels]
        img = np.zeros(n_img, dtype=IMAGE_DT)
        img["band"] = band
        img["h"] = h
        img["w"] = w
        img["pitch"] = pitch
        img["n_psf"] = npsf
        img["origin"] = origin
        img["wcs"] = wcs
        img["sky"] = sky
        img["calib"] = calib
        K = psf.shape[1]
        img["psf"][:, :K, :] = psf
        base = _ptr(pixels)
        img["pixels"] = base + 4 * np.asarray(pix_off, dtype=np.uint64)
        for name, arr in (("nbr_mean", nbr_mean), ("nbr_var", nbr_var)):
            if arr is not None:
                if not self.device:
                    arr = np.ascontiguousarray(arr, dtype=np.float32)
                self._keep.append(arr)
                off = pix_off if nbr_off is None else nbr_off
                img[name] = _ptr(arr) + 4 * np.asarray(off, dtype=np.uint64)
        # neighbour rows: nbr_pitch if given, else contiguous per image when separate offsets
        # are given, else the pixel pitch
        if nbr_pitch is not None:
            img["nbr_pitch"] = nbr_pitch
        elif nbr_off is not None:
            img["nbr_pitch"] = w
        pr = np.zeros(1, dtype=PRIOR_DT)
        pr["p_star"] = prior["p_star"]
        pr["r_mean"] = prior["r_mean"]
        pr["r_var"] = prior["r_var"]
        pr["c_mean"] = prior["c_mean"]
        pr["c_cov"] = prior["c_cov"]
        pf = np.zeros(1, dtype=PROF_DT)
        ea, ev = profiles["exp"]
        da, dv = profiles["dev"]
        pf["n_exp"], pf["n_dev"] = len(ea), len(da)
        pf["exp_amp"][0, :len(ea)] = ea
        pf["exp_var"][0, :len(ev)] = ev
        pf["dev_amp"][0, :len(da)] = da
        pf["dev_var"][0, :len(dv)] = dv
        self.offsets = np.ascontiguousarray(src_img_off, dtype=np.int64)
        self.images, self.prior, self.profiles = img, pr, pf
        self.n_sources = len(self.offsets) - 1
        self.c = CBatch(self.n_sources, MEM_DEVICE if self.device else MEM_HOST, self.offsets.ctypes.data,
                        img.ctypes.data, pr.ctypes.data, pf.ctypes.data)
        self.torch_device = pixels.device if self.device else None

    @classmethod
    def from_synth(cls, sb, nbr=None):
        """From a synth.SynthBatch (pixels host ndarray or device tensor)."""
        kw = {}
        if nbr is not None:
            kw = dict(nbr_mean=nbr[0], nbr_var=nbr[1], nbr_off=nbr[2] if len(nbr) > 2 else None)
        return cls(sb.src_img_off, sb.img_band, sb.img_h, sb.img_w, sb.img_pitch, sb.img_origin, sb.img_wcs,
                   sb.img_sky, sb.img_calib, sb.img_psf, sb.img_npsf, sb.pixels, sb.img_pix_off, sb.prior,
                   sb.profiles, **kw)

    def subset(self, idx):
        """A batch of the sources idx (in that order) sharing this batch's pixel memory, and
        the indices of their images in this batch."""
        idx = np.asarray(idx, dtype=np.int64)
        counts = self.offsets[idx + 1] - self.offsets[idx]
        img_idx = (np.repeat(self.offsets[idx] - np.concatenate([[0], np.cumsum(counts)[:-1]]), counts)
                   + np.arange(int(counts.sum())))
        b = Batch.__new__(Batch)
        b.device, b.torch_device, b._keep = self.device, self.torch_device, list(self._keep)
        b.images = np.ascontiguousarray(self.images[img_idx])
        b.prior, b.profiles = self.prior, self.profiles
        b.offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        b.n_sources = len(idx)
        b.c = CBatch(b.n_sources, self.c.mem_kind, b.offsets.ctypes.data, b.images.ctypes.data,
                     b.prior.ctypes.data, b.profiles.ctypes.data)
        return b, img_idx

    def with_nbr(self, nbr_mean, nbr_var, nbr_off):
        """This batch with per-image neighbour arrays at element offsets nbr_off (one per image,
        rows of w elements) of nbr_mean / nbr_var."""
        b = Batch.__new__(Batch)
        b.device, b.torch_device = self.device, self.torch_device
        b._keep = list(self._keep) + [nbr_mean, nbr_var]
        b.images = self.images.copy()
        off = np.asarray(nbr_off, dtype=np.uint64)
        b.images["nbr_mean"] = _ptr(nbr_mean) + 4 * off
        b.images["nbr_var"] = _ptr(nbr_var) + 4 * off
        b.images["nbr_pitch"] = b.images["w"]
        b.prior, b.profiles, b.offsets, b.n_sources = self.prior, self.profiles, self.offsets, self.n_sources
        b.c = CBatch(b.n_sources, self.c.mem_kind, b.offsets.ctypes.data, b.images.ctypes.data,
                     b.prior.ctypes.data, b.profiles.ctypes.data)
        return b

    def array(self, shape):
        """An output array of the batch's memory kind."""
        if self.device:
            import torch
            return torch.empty(shape, dtype=torch.float64, device=self.torch_device)
        return np.empty(shape, dtype=np.float64)

    def as_input(self, x, copy=False):
        """x as an array of the batch's memory kind; copy=True always returns a fresh array
        (used for the in/out parameter of the fits, so the caller's start is not overwritten)."""
        if self.device:
            import torch
            t = torch.as_tensor(np.asarray(x) if not _is_torch(x) else x, dtype=torch.float64,
                                device=self.torch_device).contiguous()
            return t.clone() if copy else t
        a = np.ascontiguousarray(x.cpu().numpy() if _is_torch(x) else x, dtype=np.float64)
        return a.copy() if copy else a


class Context:
    def __init__(self, device=0):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.celeste_ctx_create(int(device), ctypes.byref(h)))
        self._h = h
        self.device = device

    def close(self):
        if self._h:
            load().celeste_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, option, value):
        _check(load().celeste_ctx_set_option(self._h, int(option), int(value)))

    def autotune(self, batch: Batch, theta, sample_px=0, cache_path=None):
        """Time the pixel kernels' launch and tile shapes on a sample of the batch at theta and
        keep the fastest on this context (celeste_autotune).  Returns the choice as a dict."""
        th = batch.as_input(theta)
        r = TuneResult()
        self._stream(batch)
        _check(load().celeste_autotune(self._h, ctypes.byref(batch.c), _ptr(th), int(sample_px),
                                       None if cache_path is None else os.fsencode(cache_path), ctypes.byref(r)))
        return {name: getattr(r, name) for name, _ in TuneResult._fields_}

    def stats(self, reset=False):
        st = Stats()
        _check(load().celeste_ctx_get_stats(self._h, ctypes.byref(st), 1 if reset else 0))
        return {name: getattr(st, name) for name, _ in Stats._fields_}

    def _stream(self, batch):
        # Work on device tensors queued by torch must be complete before the library's
        # own (non-blocking) stream reads them; the library synchronises before returning.
        if batch.device:
            import torch
            torch.cuda.synchronize(batch.torch_device)
        return None

    def elbo_eval(self, batch: Batch, theta, want="hess"):
        """ELBO (S,), gradient (S,27) and Hessian (S,27,27) at theta (S,27); want in {value, grad, hess}."""
        S = batch.n_sources
        th = batch.as_input(theta)
        if tuple(th.shape) != (S, NP):
            raise ValueError(f"theta must have shape ({S}, {NP})")
        elbo = batch.array((S,))
        grad = batch.array((S, NP)) if want in ("grad", "hess") else None
        hess = batch.array((S, NP, NP)) if want == "hess" else None
        _check(load().celeste_elbo_eval(self._h, ctypes.byref(batch.c), _ptr(th), _ptr(elbo),
                                        _ptr(grad) if grad is not None else None,
                                        _ptr(hess) if hess is not None else None, self._stream(batch)))
        return elbo, grad, hess

    def elbo_eval_noalloc(self, batch: Batch, theta, elbo, grad=None, hess=None):
        """elbo_eval into caller-owned device tensors through the entry point that allocates
        nothing (celeste_elbo_eval_noalloc): a device batch (the library refuses host batches),
        theta (S, 27), and float64 CUDA tensors elbo (S,), grad (S, 27) or None, hess
        (S, 27, 27) or None."""
        S = batch.n_sources
        th = batch.as_input(theta)
        if tuple(th.shape) != (S, NP):
            raise ValueError(f"theta must have shape ({S}, {NP})")
        for name, t, shape in (("elbo", elbo, (S,)), ("grad", grad, (S, NP)), ("hess", hess, (S, NP, NP))):
            if t is None:
                continue
            if not (_is_torch(t) and t.is_cuda) or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous CUDA tensor of shape {shape}")
        _check(load().celeste_elbo_eval_noalloc(self._h, ctypes.byref(batch.c), _ptr(th), _ptr(elbo),
                                                _ptr(grad) if grad is not None else None,
                                                _ptr(hess) if hess is not None else None, self._stream(batch)))
        return elbo, grad, hess

    def elbo_eval_sampled(self, batch: Batch, theta, keep, keep_off, keep_prob, want="hess"):
        """Pixel-subsampled estimate of elbo_eval's results: keep (uint8) and keep_off (int64,
        n_images + 1) select 8-row blocks of each image, kept blocks weigh 1 / keep_prob."""
        S = batch.n_sources
        th = batch.as_input(theta)
        if tuple(th.shape) != (S, NP):
            raise ValueError(f"theta must have shape ({S}, {NP})")
        kp = np.ascontiguousarray(keep, dtype=np.uint8)
        ko = np.ascontiguousarray(keep_off, dtype=np.int64)
        if ko.ndim != 1 or kp.ndim != 1 or ko.size != len(batch.images) + 1 or ko[-1] != kp.size:
            raise ValueError("keep_off must hold n_images + 1 offsets ending at keep.size")
        elbo = batch.array((S,))
        grad = batch.array((S, NP)) if want in ("grad", "hess") else None
        hess = batch.array((S, NP, NP)) if want == "hess" else None
        _check(load().celeste_elbo_eval_sampled(self._h, ctypes.byref(batch.c), _ptr(th), kp.ctypes.data,
                                                ko.ctypes.data, float(keep_prob), _ptr(elbo),
                                                _ptr(grad) if grad is not None else None,
                                                _ptr(hess) if hess is not None else None, self._stream(batch)))
        return elbo, grad, hess

    def lr_covariance(self, batch: Batch, theta, u0, u_box=3.0):
        """Linear-response covariance (S, 27, 27) at theta, with the gradient and Hessian
        evaluated by the pixel sum; u0 (S, 2) are the fits' position-box centres.  Returns
        (cov, status) with status (S,) int32 on the host."""
        S = batch.n_sources
        th = batch.as_input(theta)
        uu = batch.as_input(u0)
        if tuple(th.shape) != (S, NP) or tuple(uu.shape) != (S, 2):
            raise ValueError(f"theta must have shape ({S}, {NP}) and u0 ({S}, 2)")
        cov = batch.array((S, NP, NP))
        status = np.zeros(S, dtype=np.int32)
        _check(load().celeste_lr_covariance(self._h, ctypes.byref(batch.c), _ptr(th), _ptr(uu), float(u_box),
                                            _ptr(cov), status.ctypes.data, self._stream(batch)))
        return cov, status

    def lr_covariance_from_hessian(self, theta, u0, grad, hess, u_box=3.0):
        """The same from given natural gradients (n, 27) and Hessians (n, 27, 27): NumPy arrays
        (host memory) or CUDA tensors (device memory), all of one kind."""
        dev = _is_torch(theta) and theta.is_cuda
        if dev:
            import torch
            arrs = [x.to(torch.float64).contiguous() for x in (theta, u0, grad, hess)]
            torch.cuda.synchronize(arrs[0].device)
        else:
            arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (theta, u0, grad, hess)]
        th, uu, g, H = arrs
        n = th.shape[0]
        if tuple(th.shape) != (n, NP) or tuple(uu.shape) != (n, 2) or tuple(g.shape) != (n, NP) \
                or tuple(H.shape) != (n, NP, NP):
            raise ValueError("theta (n, 27), u0 (n, 2), grad (n, 27), hess (n, 27, 27) expected")
        if dev:
            import torch
            cov = torch.empty((n, NP, NP), dtype=torch.float64, device=th.device)
        else:
            cov = np.empty((n, NP, NP), dtype=np.float64)
        status = np.zeros(n, dtype=np.int32)
        _check(load().celeste_lr_covariance_from_hessian(self._h, n, MEM_DEVICE if dev else MEM_HOST, _ptr(th),
                                                         _ptr(uu), float(u_box), _ptr(g), _ptr(H), _ptr(cov),
                                                         status.ctypes.data, None))
        return cov, status

    def newton_fit(self, batch: Batch, theta0, opts=None):
        if batch.n_sources != 1:
            raise ValueError("newton_fit takes one source")
        th = batch.as_input(np.asarray(theta0).reshape(1, NP) if not _is_torch(theta0) else theta0.reshape(1, NP),
                            copy=True)
        res = np.zeros(1, dtype=RESULT_DT)
        o = opts if opts is not None else default_opts()
        self._stream(batch)
        _check(load().celeste_newton_fit(self._h, ctypes.byref(batch.c), _ptr(th), ctypes.byref(o),
                                         res.ctypes.data))
        return th, res[0]

    def set_surrogate(self, net):
        _check(load().celeste_ctx_set_surrogate(self._h, net._h if net is not None else None))
        self._net = net

    def make_patches(self, batch: Batch, theta):
        """Network inputs (torch BF16 on the device, S x 5 x 32 x 32) around theta's positions."""
        import torch
        th = batch.as_input(theta)
        dev = batch.torch_device if batch.device else torch.device("cuda", self.device)
        out = torch.empty((batch.n_sources, 5, 32, 32), dtype=torch.bfloat16, device=dev)
        self._stream(batch)
        _check(load().celeste_make_patches(self._h, ctypes.byref(batch.c), _ptr(th), out.data_ptr()))
        return out

    def start(self, batch: Batch, theta0, opts=None):
        """The start a fit with these options would use, and its ELBO (no fitting)."""
        th = batch.as_input(theta0, copy=True)
        el = batch.array((batch.n_sources,))
        o = opts if opts is not None else default_opts()
        self._stream(batch)
        _check(load().celeste_start(self._h, ctypes.byref(batch.c), _ptr(th), ctypes.byref(o), _ptr(el)))
        return th, el

    def render_fields(self, batch: Batch, theta, img_field, n_fields, height, width, out=None):
        """Expected counts and variance of all sources summed into the field images (device)."""
        import torch
        th = batch.as_input(theta)
        if out is None:
            out = (torch.empty(n_fields * height * width, dtype=torch.float32, device=batch.torch_device),
                   torch.empty(n_fields * height * width, dtype=torch.float32, device=batch.torch_device))
        f, keep = self._fields(img_field, n_fields, height, width, out)
        self._stream(batch)
        _check(load().celeste_render_fields(self._h, ctypes.byref(batch.c), _ptr(th), ctypes.byref(f)))
        return out

    def neighbour_arrays(self, batch: Batch, theta, img_field, n_fields, height, width, fields, nbr_off, nbr_mean,
                         nbr_var):
        th = batch.as_input(theta)
        f, keep = self._fields(img_field, n_fields, height, width, fields)
        off = np.ascontiguousarray(nbr_off, dtype=np.int64)
        self._stream(batch)
        _check(load().celeste_neighbour_arrays(self._h, ctypes.byref(batch.c), _ptr(th), ctypes.byref(f),
                                               off.ctypes.data, _ptr(nbr_mean), _ptr(nbr_var)))

    def update_fields(self, batch: Batch, theta_old, theta_new, img_field, n_fields, height, width, fields):
        """Move the rendered fields of the batch's sources (one colour) from theta_old to theta_new."""
        to, tn = batch.as_input(theta_old), batch.as_input(theta_new)
        f, keep = self._fields(img_field, n_fields, height, width, fields)
        self._stream(batch)
        _check(load().celeste_update_fields(self._h, ctypes.byref(batch.c), _ptr(to), _ptr(tn), ctypes.byref(f)))

    def field_elbo(self, batch: Batch, theta, img_field, n_fields, height, width, fields, field_pixels, field_sky):
        """Joint ELBO of the field at theta (fields rendered at theta)."""
        th = batch.as_input(theta)
        f, keep = self._fields(img_field, n_fields, height, width, fields)
        sky = np.ascontiguousarray(field_sky, dtype=np.float64)
        out = ctypes.c_double()
        self._stream(batch)
        _check(load().celeste_field_elbo(self._h, ctypes.byref(batch.c), _ptr(th), ctypes.byref(f),
                                         _ptr(field_pixels), sky.ctypes.data, ctypes.byref(out)))
        return out.value

    @staticmethod
    def _fields(img_field, n_fields, height, width, arrays):
        imf = np.ascontiguousarray(img_field, dtype=np.int32)
        f = CFields(int(n_fields), int(height), int(width), 0, imf.ctypes.data, _ptr(arrays[0]), _ptr(arrays[1]))
        return f, imf

    def batch_fit_sampled(self, batch: Batch, theta0, keep, keep_off, keep_prob, switch_rtol=1e-5, opts=None):
        """batch_fit with a pixel-subsampled early phase (celeste_batch_fit_sampled): keep (uint8)
        and keep_off (int64, n_images + 1) select each image's kept 8-row blocks."""
        S = batch.n_sources
        th = batch.as_input(theta0, copy=True)
        if tuple(th.shape) != (S, NP):
            raise ValueError(f"theta0 must have shape ({S}, {NP})")
        kp = np.ascontiguousarray(keep, dtype=np.uint8)
        ko = np.ascontiguousarray(keep_off, dtype=np.int64)
        if ko.ndim != 1 or kp.ndim != 1 or ko.size != len(batch.images) + 1 or ko[-1] != kp.size:
            raise ValueError("keep_off must hold n_images + 1 offsets ending at keep.size")
        res = np.zeros(S, dtype=RESULT_DT)
        o = opts if opts is not None else default_opts()
        _check(load().celeste_batch_fit_sampled(self._h, ctypes.byref(batch.c), _ptr(th), ctypes.byref(o),
                                                kp.ctypes.data, ko.ctypes.data, float(keep_prob),
                                                float(switch_rtol), res.ctypes.data, self._stream(batch)))
        return th, res

    def lbfgs_fit(self, batch: Batch, theta0, opts=None):
        """L-BFGS fit of every source (celeste_lbfgs_fit); returns (theta, results) like batch_fit
        (iters = accepted steps, n_full_evals = value+gradient evaluations)."""
        S = batch.n_sources
        th = batch.as_input(theta0, copy=True)
        if tuple(th.shape) != (S, NP):
            raise ValueError(f"theta0 must have shape ({S}, {NP})")
        res = np.zeros(S, dtype=RESULT_DT)
        o = opts if opts is not None else default_lbfgs_opts()
        _check(load().celeste_lbfgs_fit(self._h, ctypes.byref(batch.c), _ptr(th), ctypes.byref(o),
                                        res.ctypes.data, self._stream(batch)))
        return th, res

    def batch_fit(self, batch: Batch, theta0, opts=None):
        S = batch.n_sources
        th = batch.as_input(theta0, copy=True)
        if tuple(th.shape) != (S, NP):
            raise ValueError(f"theta0 must have shape ({S}, {NP})")
        res = np.zeros(S, dtype=RESULT_DT)
        o = opts if opts is not None else default_opts()
        _check(load().celeste_batch_fit(self._h, ctypes.byref(batch.c), _ptr(th), ctypes.byref(o),
                                        res.ctypes.data, self._stream(batch)))
        return th, res


def theta_to_psi(theta, u0, u_box=3.0):
    theta = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1, NP)
    u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(-1, 2)
    out = np.empty_like(theta)
    _check(load().celeste_theta_to_psi(theta.ctypes.data, u0.ctypes.data, theta.shape[0], u_box, out.ctypes.data))
    return out


def psi_to_theta(psi, u0, u_box=3.0):
    psi = np.ascontiguousarray(psi, dtype=np.float64).reshape(-1, NP)
    u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(-1, 2)
    out = np.empty_like(psi)
    _check(load().celeste_psi_to_theta(psi.ctypes.data, u0.ctypes.data, psi.shape[0], u_box, out.ctypes.data))
    return out


class Net:
    """The surrogate initialiser network on a context's device (weights in FP32 + BF16)."""

    def __init__(self, ctx: Context, params, psi_mean, psi_std):
        lib = load()
        params = np.ascontiguousarray(params, dtype=np.float32)
        mean = np.ascontiguousarray(psi_mean, dtype=np.float32)
        sd = np.ascontiguousarray(psi_std, dtype=np.float32)
        h = ctypes.c_void_p()
        _check(lib.celeste_net_create(ctx._h, params.ctypes.data, params.size, mean.ctypes.data, sd.ctypes.data,
                                      ctypes.byref(h)))
        self._h = h
        self.psi_mean, self.psi_std = mean, sd

    @staticmethod
    def num_params():
        return int(load().celeste_net_num_params())

    def close(self):
        if self._h:
            load().celeste_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        out = np.empty(self.num_params(), dtype=np.float32)
        _check(load().celeste_net_get_params(self._h, out.ctypes.data))
        return out

    def loss_grad(self, x, t, want_grad=True):
        import torch
        torch.cuda.synchronize()
        loss = ctypes.c_float()
        g = np.empty(self.num_params(), dtype=np.float32) if want_grad else None
        _check(load().celeste_net_loss_grad(self._h, x.data_ptr(), t.data_ptr(), int(x.shape[0]),
                                            ctypes.byref(loss), g.ctypes.data if g is not None else None))
        return float(loss.value), g

    def forward(self, x):
        import torch
        torch.cuda.synchronize()
        y = torch.empty((x.shape[0], 27), dtype=torch.float32, device=x.device)
        _check(load().celeste_net_forward(self._h, x.data_ptr(), int(x.shape[0]), y.data_ptr()))
        return y

    def train(self, x, t, orders, batch=256, lr=1e-3):
        import torch
        torch.cuda.synchronize()
        epochs = int(orders.shape[0])
        losses = np.zeros(epochs, dtype=np.float32)
        _check(load().celeste_net_train(self._h, x.data_ptr(), t.data_ptr(), int(x.shape[0]), orders.data_ptr(),
                                        epochs, int(batch), float(lr), losses.ctypes.data))
        return losses
