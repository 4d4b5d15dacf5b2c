"""ctypes binding of libpcmd.so (include/pcmd.h): argument marshalling only.

Device arrays are torch tensors on the context's GPU; the binding passes their data pointers
and the current HIP stream.  Every step of the forward model runs in the library's kernels.
If the library is missing the binding raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcmd.so")

MAX_BANDS = 4
MAX_ISO = 512

OK, E_INVAL, E_HIP, E_NOMEM, E_UNSUPPORTED, E_PTRS_RETRY = 0, -1, -2, -3, -4, -5
SFH = {"ssp": 0, "const": 1, "tau": 2, "dtau": 3, "nonparam": 4}
MDF = {"single": 0, "gauss": 1}
DUST_NONE, DUST_SCREEN, DUST_LOGNORMAL = 0, 1, 2
CONV_AUTO, CONV_DIRECT, CONV_FFT = 0, 1, 2
NOISE_NONE, NOISE_GAUSS_MAG, NOISE_SHOT = 0, 1, 2
SAMPLER_POINT, SAMPLER_BLOCK, SAMPLER_HYBRID = 0, 1, 2
LL_POISSON, LL_GAUSS_PAPER, LL_GAUSS_LITERAL = 0, 1, 2
LL_ACCUMULATE = 0x100  # OR-ed into mode: add to out instead of storing
TIMER_SAMPLE, TIMER_CONV, TIMER_HESS, TIMER_BATCH, TIMER_GEMM = 0, 1, 2, 3, 4

D4 = C.c_double * MAX_BANDS


class PcmdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pcmd error {code}: {msg}")
        self.code = code
        self.msg = msg


class IsoSet(C.Structure):
    _fields_ = [("n_iso", C.c_int32), ("n_age", C.c_int32), ("n_feh", C.c_int32),
                ("age_edges", C.POINTER(C.c_double)), ("feh_grid", C.POINTER(C.c_double)),
                ("iso_age", C.POINTER(C.c_int32)), ("iso_feh", C.POINTER(C.c_int32))]


class ModelS(C.Structure):
    _fields_ = [("sfh", C.c_int32), ("mdf", C.c_int32), ("ssp_age_index", C.c_int32), ("feh_index", C.c_int32),
                ("log_npix", C.c_double), ("tau_gyr", C.c_double), ("feh_mu", C.c_double),
                ("feh_sigma", C.c_double), ("mdf_prune", C.c_double), ("log_sfh", C.POINTER(C.c_double))]


class GridS(C.Structure):
    _fields_ = [("n_entries", C.c_int32), ("n_iso", C.c_int32), ("iso_of_entry", C.c_void_p),
                ("imf_w", C.c_void_p), ("iso_imf_sum", C.POINTER(C.c_double))]


class IsoS(C.Structure):
    _fields_ = [("n_entries", C.c_int32), ("n_bands", C.c_int32), ("lam", C.c_void_p), ("flux", C.c_void_p)]


class ObsS(C.Structure):
    _fields_ = [("nim", C.c_int32), ("dust_model", C.c_int32), ("seed", C.c_uint64), ("dmod", C.c_double),
                ("dust_mu", C.c_double), ("dust_sigma", C.c_double), ("dust_frac", C.c_double),
                ("dust_R", D4), ("psf_k", C.c_int32), ("conv_path", C.c_int32), ("psf", C.c_void_p),
                ("noise_model", C.c_int32), ("psf_grid", C.c_int32), ("noise_sigma_mag", D4), ("exptime", D4),
                ("zp", D4), ("sky", D4), ("sampler", C.c_int32), ("pad_", C.c_int32)]


class DebugS(C.Structure):
    _fields_ = [("counts", C.c_void_p), ("reddened", C.c_void_p), ("px0", C.c_int64), ("px1", C.c_int64),
                ("flux_pre", C.c_void_p), ("flux_psf", C.c_void_p)]


class JobS(C.Structure):
    _fields_ = [("iso", IsoS), ("obs", ObsS)]


class TuningS(C.Structure):
    _fields_ = [("wg_per_cu", C.c_int32), ("order", C.c_int32)]


MLP_MAX_LAYERS = 8


class MlpS(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("dims", C.c_int32 * (MLP_MAX_LAYERS + 1)), ("master", C.c_void_p),
                ("adam_m", C.c_void_p), ("adam_v", C.c_void_p), ("w_bf16", C.c_void_p), ("wt_bf16", C.c_void_p)]


class HessGridS(C.Structure):
    _fields_ = [("x0", C.c_double), ("dx", C.c_double), ("y0", C.c_double), ("dy", C.c_double),
                ("nx", C.c_int32), ("ny", C.c_int32), ("b_blue", C.c_int32), ("b_red", C.c_int32),
                ("b_mag", C.c_int32), ("pad_", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libpcmd.so (raises OSError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is not built: run `python -m paper_1904_00011_amd.build`")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "pcmd_create": (C.c_int, [C.POINTER(vp), C.c_int]),
        "pcmd_destroy": (None, [vp]),
        "pcmd_last_error": (C.c_char_p, [vp]),
        "pcmd_sync": (C.c_int, [vp, vp]),
        "pcmd_version": (C.c_char_p, []),
        "pcmd_grid_prepare": (C.c_int, [i32, i32, vp, vp, vp, i32, dbl, vp, vp, i32, vp]),
        "pcmd_iso_weights": (C.c_int, [C.POINTER(ModelS), C.POINTER(IsoSet), vp, C.POINTER(dbl)]),
        "pcmd_lmax_ceiling": (C.c_int, [vp, i64, C.POINTER(dbl)]),
        "pcmd_cap_loglikes": (C.c_int, [vp, i64, dbl, vp]),
        "pcmd_nested_weights": (C.c_int, [vp, vp, i64, vp]),
        "pcmd_remaining_evidence": (C.c_int, [vp, vp, i64, dbl, dbl, C.POINTER(dbl)]),
        "pcmd_effective_sample_size": (C.c_int, [vp, i64, C.POINTER(dbl)]),
        "pcmd_entries": (C.c_int, [vp, C.POINTER(GridS), vp, dbl, vp, vp]),
        "pcmd_simulate": (C.c_int, [vp, C.POINTER(IsoS), C.POINTER(ObsS), vp, C.POINTER(DebugS), vp]),
        "pcmd_hess": (C.c_int, [vp, vp, i32, i64, C.POINTER(HessGridS), vp, vp, vp]),
        "pcmd_loglike": (C.c_int, [vp, vp, vp, i32, vp, vp, i32, dbl, vp, vp]),
        "pcmd_batch_run": (C.c_int, [vp, i32, C.POINTER(JobS), C.POINTER(HessGridS), vp, vp, i32, dbl, vp, vp, i32, vp]),
        "pcmd_batch_set_tuning": (C.c_int, [vp, C.POINTER(TuningS)]),
        "pcmd_batch_get_tuning": (C.c_int, [vp, C.POINTER(TuningS)]),
        "pcmd_batch_autotune": (C.c_int, [vp, i32, C.POINTER(JobS), C.POINTER(HessGridS), vp, vp, i32, dbl, vp,
                                          C.POINTER(TuningS), vp, C.POINTER(i32), vp]),
        "pcmd_mlp_param_count": (C.c_int64, [C.POINTER(i32), i32]),
        "pcmd_mlp_weight_count": (C.c_int64, [C.POINTER(i32), i32]),
        "pcmd_mlp_refresh": (C.c_int, [vp, C.POINTER(MlpS), vp]),
        "pcmd_mlp_forward": (C.c_int, [vp, C.POINTER(MlpS), i32, vp, vp, vp]),
        "pcmd_mlp_train_step": (C.c_int, [vp, C.POINTER(MlpS), i32, vp, vp, C.c_float, i32, vp, vp, i32, vp]),
        "pcmd_mlp_backward": (C.c_int, [vp, C.POINTER(MlpS), i32, vp, vp, vp, i64, vp, vp, vp]),
        "pcmd_mlp_adam": (C.c_int, [vp, C.POINTER(MlpS), vp, C.c_float, i32, vp]),
        "pcmd_mlp_loss": (C.c_int, [vp, C.POINTER(MlpS), i32, vp, vp, vp, i64, vp, vp]),
        "pcmd_log_hess_target": (C.c_int, [vp, vp, i32, i32, vp, vp]),
        "pcmd_surrogate_loglike": (C.c_int, [vp, vp, i32, i32, vp, vp, vp]),
        "pcmd_gemm_bf16": (C.c_int, [vp, i32, i32, i32, vp, i32, i32, vp, i32, i32, vp, i32, vp]),
        "pcmd_timer_enable": (C.c_int, [vp, C.c_int]),
        "pcmd_timer_read": (C.c_int, [vp, C.c_int, C.POINTER(dbl), C.POINTER(i64), C.POINTER(dbl)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _np_ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------------------------------------
# host helpers (a0)
# ---------------------------------------------------------------------------------------------

IMF_POWER_LAW, IMF_KROUPA = 0, 1


def grid_prepare(iso_of_entry, mass, absmag, alpha: float = 2.35, imf: str = "salpeter", n_iso: int | None = None):
    """IMF weight per point and FP32 star flux per band (host); with n_iso also the IMF weight
    summed over each isochrone's points: (imf_w, flux) or (imf_w, flux, iso_imf_sum)."""
    lib = load()
    iso = np.ascontiguousarray(iso_of_entry, dtype=np.int32)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    absmag = np.ascontiguousarray(absmag, dtype=np.float64)
    B, E = absmag.shape
    w = np.empty(E, dtype=np.float64)
    f = np.empty((B, E), dtype=np.float32)
    sums = None if n_iso is None else np.empty(int(n_iso), dtype=np.float64)
    kind = IMF_KROUPA if imf == "kroupa" else IMF_POWER_LAW
    rc = lib.pcmd_grid_prepare(E, B, iso.ctypes.data, mass.ctypes.data, absmag.ctypes.data, kind, float(alpha),
                               w.ctypes.data, f.ctypes.data, 0 if n_iso is None else int(n_iso),
                               None if sums is None else sums.ctypes.data)
    if rc != OK:
        raise PcmdError(rc, "pcmd_grid_prepare rejected its arguments")
    return (w, f) if sums is None else (w, f, sums)


def model_struct(model, keep: list):
    log_sfh = None
    if getattr(model, "sfh", "ssp") == "nonparam":
        arr = np.ascontiguousarray(model.log_sfh, dtype=np.float64)
        keep.append(arr)
        log_sfh = _np_ptr(arr, C.c_double)
    return ModelS(SFH[model.sfh], MDF[model.mdf], int(getattr(model, "ssp_age_index", 0)),
                  int(getattr(model, "feh_index", 0)), float(getattr(model, "log_npix", 2.0)),
                  float(getattr(model, "tau_gyr", 1.0)), float(getattr(model, "feh_mu", 0.0)),
                  float(getattr(model, "feh_sigma", 0.2)), float(getattr(model, "mdf_prune", 0.01)), log_sfh)


def isoset_struct(grid, keep: list):
    arrs = [np.ascontiguousarray(grid.age_edges, dtype=np.float64), np.ascontiguousarray(grid.feh_grid, dtype=np.float64),
            np.ascontiguousarray(grid.age_index, dtype=np.int32), np.ascontiguousarray(grid.feh_index, dtype=np.int32)]
    keep.extend(arrs)
    return IsoSet(int(grid.n_iso), len(arrs[0]) - 1, len(arrs[1]), _np_ptr(arrs[0], C.c_double),
                  _np_ptr(arrs[1], C.c_double), _np_ptr(arrs[2], C.c_int32), _np_ptr(arrs[3], C.c_int32))


def iso_weights(model, grid):
    """Per-isochrone SFH x MDF weights and Npix (host)."""
    lib = load()
    keep = []
    ms = model_struct(model, keep)
    ss = isoset_struct(grid, keep)
    w = np.empty(grid.n_iso, dtype=np.float64)
    npix = C.c_double(0.0)
    rc = lib.pcmd_iso_weights(C.byref(ms), C.byref(ss), w.ctypes.data, C.byref(npix))
    if rc != OK:
        raise PcmdError(rc, "pcmd_iso_weights rejected its arguments")
    return w, npix.value


def obs_struct(obs, B: int, psf_tensor=None, conv_path: int = CONV_AUTO):
    def arr(v, fill):
        vals = list(v)[:MAX_BANDS] if v is not None else []
        vals = vals + [fill] * (MAX_BANDS - len(vals))
        return D4(*[float(x) for x in vals])
    K = 1 if psf_tensor is None else int(psf_tensor.shape[-1])
    # [B][K][K]: one PSF per band; [B][16][K][K]: the 4 x 4 grid of sub-pixel PSFs
    grid = 4 if psf_tensor is not None and psf_tensor.dim() == 4 else 1
    return ObsS(int(obs.nim), int(obs.dust_model), int(obs.seed) & 0xFFFFFFFFFFFFFFFF, float(obs.dmod),
                float(obs.dust_mu), float(obs.dust_sigma), float(obs.dust_frac), arr(obs.dust_R, 0.0), K,
                int(conv_path), _ptr(psf_tensor), int(obs.noise_model), grid, arr(obs.noise_sigma_mag, 0.0),
                arr(obs.exptime, 1.0), arr(obs.zp, 0.0), arr(obs.sky, 0.0), int(getattr(obs, "sampler", SAMPLER_POINT)),
                0)


def hess_grid_struct(g: dict, bands=(0, 1, 1)):
    return HessGridS(float(g["x0"]), float(g["dx"]), float(g["y0"]), float(g["dy"]), int(g["nx"]), int(g["ny"]),
                     int(bands[0]), int(bands[1]), int(bands[2]), 0)


# ---------------------------------------------------------------------------------------------
# context
# ---------------------------------------------------------------------------------------------

class Context:
    """One library context on one GPU (owns the library's scratch)."""

    def __init__(self, device: int = 0):
        self.lib = load()
        h = C.c_void_p()
        rc = self.lib.pcmd_create(C.byref(h), int(device))
        if rc != OK:
            raise PcmdError(rc, f"pcmd_create(device={device}) failed")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self.lib.pcmd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, name: str):
        if rc != OK:
            raise PcmdError(rc, f"{name}: {self.lib.pcmd_last_error(self.h).decode()}")

    def timer_enable(self, on: bool = True):
        self._check(self.lib.pcmd_timer_enable(self.h, int(bool(on))), "pcmd_timer_enable")

    def timer_read(self, which: int):
        """(total_ms, launches, units) of the recorded launches of kernel `which`."""
        ms, n, u = C.c_double(), C.c_int64(), C.c_double()
        self._check(self.lib.pcmd_timer_read(self.h, int(which), C.byref(ms), C.byref(n), C.byref(u)),
                    "pcmd_timer_read")
        return ms.value, n.value, u.value

    def sync(self, stream=None):
        self._check(self.lib.pcmd_sync(self.h, _stream(stream)), "pcmd_sync")

    def entries(self, n_entries: int, iso_of_entry_dev, imf_w_dev, iso_imf_sum, iso_w, npix, lam_out, stream=None):
        iso_imf_sum = np.ascontiguousarray(iso_imf_sum, dtype=np.float64)
        iso_w = np.ascontiguousarray(iso_w, dtype=np.float64)
        g = GridS(int(n_entries), len(iso_w), _ptr(iso_of_entry_dev), _ptr(imf_w_dev), _np_ptr(iso_imf_sum, C.c_double))
        self._check(self.lib.pcmd_entries(self.h, C.byref(g), iso_w.ctypes.data, float(npix), _ptr(lam_out),
                                          _stream(stream)), "pcmd_entries")

    def simulate(self, lam, flux, obs, mags_out, psf=None, conv_path: int = CONV_AUTO, counts=None, reddened=None,
                 px0: int = 0, px1: int = 0, flux_pre=None, flux_psf=None, stream=None):
        B, E = int(flux.shape[0]), int(flux.shape[1])
        iso = IsoS(E, B, _ptr(lam), _ptr(flux))
        o = obs_struct(obs, B, psf, conv_path)
        dbg = DebugS(_ptr(counts), _ptr(reddened), int(px0), int(px1), _ptr(flux_pre), _ptr(flux_psf))
        self._check(self.lib.pcmd_simulate(self.h, C.byref(iso), C.byref(o), _ptr(mags_out), C.byref(dbg),
                                           _stream(stream)), "pcmd_simulate")

    def hess(self, mags, n_bands: int, n_px: int, grid: dict, hess_out, mom_out, bands=(0, 1, 1), stream=None):
        g = hess_grid_struct(grid, bands)
        self._check(self.lib.pcmd_hess(self.h, _ptr(mags), int(n_bands), int(n_px), C.byref(g), _ptr(hess_out),
                                       _ptr(mom_out), _stream(stream)), "pcmd_hess")

    def loglike(self, h_model, h_data, mom_model, mom_data, out, mode: int = LL_POISSON, eps: float = 0.01,
                stream=None):
        n = int(h_model.numel())
        self._check(self.lib.pcmd_loglike(self.h, _ptr(h_model), _ptr(h_data), n, _ptr(mom_model), _ptr(mom_data),
                                          int(mode), float(eps), _ptr(out), _stream(stream)), "pcmd_loglike")

    # -------------------------------------------------------------------------------------
    # batched evaluation
    # -------------------------------------------------------------------------------------
    @staticmethod
    def _jobs_array(jobs):
        """jobs: sequence of dicts with lam, flux (device tensors), obs, psf (device tensor or None),
        conv_path."""
        arr = (JobS * len(jobs))()
        for k, j in enumerate(jobs):
            flux = j["flux"]
            B, E = int(flux.shape[0]), int(flux.shape[1])
            arr[k].iso = IsoS(E, B, _ptr(j["lam"]), _ptr(flux))
            arr[k].obs = obs_struct(j["obs"], B, j.get("psf"), j.get("conv_path", CONV_DIRECT))
        return arr

    def batch_run(self, jobs, grid: dict, hess_data, mom_data, logl_out, mode: int = LL_POISSON, eps: float = 0.01,
                  hess_out=None, use_graph: bool = False, bands=(0, 1, 1), stream=None):
        arr = self._jobs_array(jobs)
        g = hess_grid_struct(grid, bands)
        self._check(self.lib.pcmd_batch_run(self.h, len(jobs), arr, C.byref(g), _ptr(hess_data), _ptr(mom_data),
                                            int(mode), float(eps), _ptr(logl_out), _ptr(hess_out), int(bool(use_graph)),
                                            _stream(stream)), "pcmd_batch_run")

    def batch_set_tuning(self, wg_per_cu: int, order: int):
        t = TuningS(int(wg_per_cu), int(order))
        self._check(self.lib.pcmd_batch_set_tuning(self.h, C.byref(t)), "pcmd_batch_set_tuning")

    def batch_get_tuning(self):
        t = TuningS()
        self._check(self.lib.pcmd_batch_get_tuning(self.h, C.byref(t)), "pcmd_batch_get_tuning")
        return t.wg_per_cu, t.order

    def batch_autotune(self, jobs, grid: dict, hess_data, mom_data, logl_out, mode: int = LL_POISSON,
                       eps: float = 0.01, bands=(0, 1, 1), stream=None):
        """Returns ((wg_per_cu, order), [ms per candidate])."""
        arr = self._jobs_array(jobs)
        g = hess_grid_struct(grid, bands)
        best = TuningS()
        ms = (C.c_double * 8)()
        n = C.c_int32(0)
        self._check(self.lib.pcmd_batch_autotune(self.h, len(jobs), arr, C.byref(g), _ptr(hess_data), _ptr(mom_data),
                                                 int(mode), float(eps), _ptr(logl_out), C.byref(best), ms, C.byref(n),
                                                 _stream(stream)), "pcmd_batch_autotune")
        return (best.wg_per_cu, best.order), [ms[i] for i in range(n.value)]

    # -------------------------------------------------------------------------------------
    # surrogate network
    # -------------------------------------------------------------------------------------
    def mlp_refresh(self, net, stream=None):
        self._check(self.lib.pcmd_mlp_refresh(self.h, C.byref(net), _stream(stream)), "pcmd_mlp_refresh")

    def mlp_forward(self, net, x, y, stream=None):
        self._check(self.lib.pcmd_mlp_forward(self.h, C.byref(net), int(x.shape[0]), _ptr(x), _ptr(y), _stream(stream)),
                    "pcmd_mlp_forward")

    def mlp_train_step(self, net, x, t, lr: float, step: int, loss_out=None, grad_out=None, apply_update=True,
                       stream=None):
        self._check(self.lib.pcmd_mlp_train_step(self.h, C.byref(net), int(x.shape[0]), _ptr(x), _ptr(t), float(lr),
                                                 int(step), _ptr(loss_out), _ptr(grad_out), int(bool(apply_update)),
                                                 _stream(stream)), "pcmd_mlp_train_step")

    def mlp_backward(self, net, x, t, grad_out, rows=None, loss_out=None, n: int | None = None, stream=None):
        """Gradient of one batch: the rows `rows` (int32 device vector) of x and t, or all of x."""
        nb = int(rows.shape[0]) if rows is not None else int(x.shape[0]) if n is None else int(n)
        self._check(self.lib.pcmd_mlp_backward(self.h, C.byref(net), nb, _ptr(x), _ptr(t), _ptr(rows), int(x.shape[0]),
                                               _ptr(loss_out), _ptr(grad_out), _stream(stream)), "pcmd_mlp_backward")

    def mlp_adam(self, net, grad, lr: float, step: int, stream=None):
        self._check(self.lib.pcmd_mlp_adam(self.h, C.byref(net), _ptr(grad), float(lr), int(step), _stream(stream)),
                    "pcmd_mlp_adam")

    def mlp_loss(self, net, x, t, mse_out, rows=None, stream=None):
        """Mean squared error over the rows `rows` of x and t (all rows by default) into mse_out."""
        n = int(rows.shape[0]) if rows is not None else int(x.shape[0])
        self._check(self.lib.pcmd_mlp_loss(self.h, C.byref(net), n, _ptr(x), _ptr(t), _ptr(rows), int(x.shape[0]),
                                           _ptr(mse_out), _stream(stream)), "pcmd_mlp_loss")

    def log_hess_target(self, hess, out, stream=None):
        n, nb = int(hess.shape[0]), int(hess.shape[1])
        self._check(self.lib.pcmd_log_hess_target(self.h, _ptr(hess), n, nb, _ptr(out), _stream(stream)),
                    "pcmd_log_hess_target")

    def surrogate_loglike(self, y, hess_data, out, stream=None):
        n, nb = int(y.shape[0]), int(y.shape[1])
        self._check(self.lib.pcmd_surrogate_loglike(self.h, _ptr(y), n, nb, _ptr(hess_data), _ptr(out), _stream(stream)),
                    "pcmd_surrogate_loglike")

    def gemm_bf16(self, A, B, C_out, a_trans=False, b_trans=False, stream=None):
        """C[M][N] = sum_k A(m,k) B(n,k) with A, B torch bfloat16 tensors (2-D, contiguous)."""
        M = int(A.shape[1] if a_trans else A.shape[0])
        K = int(A.shape[0] if a_trans else A.shape[1])
        N = int(B.shape[1] if b_trans else B.shape[0])
        self._check(self.lib.pcmd_gemm_bf16(self.h, M, N, K, _ptr(A), int(A.shape[1]), int(bool(a_trans)), _ptr(B),
                                            int(B.shape[1]), int(bool(b_trans)), _ptr(C_out), int(C_out.shape[1]),
                                            _stream(stream)), "pcmd_gemm_bf16")


def mlp_param_count(dims) -> int:
    arr = (C.c_int32 * len(dims))(*dims)
    return int(load().pcmd_mlp_param_count(arr, len(dims) - 1))


def mlp_weight_count(dims) -> int:
    arr = (C.c_int32 * len(dims))(*dims)
    return int(load().pcmd_mlp_weight_count(arr, len(dims) - 1))

