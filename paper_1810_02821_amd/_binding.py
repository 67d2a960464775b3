"""ctypes binding of libmf (include/mf.h).  Argument marshalling only: every
step of the messenger sweep runs in the library's HIP kernels.  Torch supplies
device memory (tensors on the GPU) and the stream (the current torch stream).
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmf.so")

MF_OK = 0
MF_ERR_NOT_CONVERGED = 5
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported size", 3: "out of memory",
          4: "device error", 5: "not converged", 6: "non-finite value"}
MF_PK_POWERLAW, MF_PK_BANDS = 0, 1
FORMS = {"auto": 0, "persistent": 1, "streamed": 2, "plain": 3}
STORAGES = {"fp32": 0, "fp16": 1, "bf16": 2}
MF_FLAG_AUTOTUNE = 1
MF_FLAG_GRAPH = 2
MF_FLAG_STREAMED_SOLVE = 4
MF_FLAG_INF_AS_1E8 = 8


class MFError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class NotConverged(MFError):
    pass


class _Spectrum(C.Structure):
    _fields_ = [("kind", C.c_int32), ("amp", C.c_double), ("k0", C.c_double), ("n", C.c_double),
                ("n_bands", C.c_int32), ("band_edges", C.POINTER(C.c_double)),
                ("band_amps", C.POINTER(C.c_double))]


class _Problem(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("noise_var", C.POINTER(C.c_float)),
                ("spectrum", _Spectrum), ("response", C.POINTER(C.c_float))]


class _Schedule(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("lam", C.POINTER(C.c_double)),
                ("sweeps", C.POINTER(C.c_int32)), ("tol", C.c_double),
                ("max_sweeps", C.c_int32), ("check_every", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("converged", C.c_int32), ("residual", C.c_double)]

    def __repr__(self):
        return f"Info(sweeps={self.sweeps}, converged={bool(self.converged)}, residual={self.residual:.3e})"


class _SampleArgs(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("chains_per_problem", C.c_int32), ("burn_in", C.c_int32),
                ("n_samples", C.c_int32), ("thin", C.c_int32), ("sweep_offset", C.c_int64),
                ("init_scale", C.c_float), ("form", C.c_int32), ("storage", C.c_int32),
                ("check_finite", C.c_int32), ("cooling", C.POINTER(_Schedule))]


class _SpectrumArgs(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("chains_per_problem", C.c_int32), ("burn_in", C.c_int32),
                ("n_samples", C.c_int32), ("thin", C.c_int32), ("sweeps_per_draw", C.c_int32),
                ("prior_dof", C.c_int32), ("prior_beta", C.c_double), ("iteration_offset", C.c_int64),
                ("init_scale", C.c_float), ("check_finite", C.c_int32)]


class _ShearArgs(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("chains_per_problem", C.c_int32), ("burn_in", C.c_int32),
                ("n_samples", C.c_int32), ("thin", C.c_int32), ("sweep_offset", C.c_int64),
                ("b_ratio", C.c_float), ("check_finite", C.c_int32)]


class _Reserve(C.Structure):
    _fields_ = [("calls", C.c_uint32), ("chains_per_problem", C.c_int32), ("storage", C.c_int32),
                ("unrolled_sweeps", C.c_int32), ("checkpoint_every", C.c_int32)]


RESERVE = {"solve": 1, "sample": 2, "spectrum": 4, "shear": 8, "unrolled": 16, "moments": 32}


EXPORTS = ["mf_plan_create", "mf_plan_destroy", "mf_plan_reserve", "mf_plan_set_spectrum", "mf_plan_pixel_offset",
           "mf_plan_tau", "mf_plan_total_bands", "mf_wiener", "mf_sample", "mf_wiener_backward",
           "mf_wiener_backward_unrolled", "mf_band_power", "mf_plan_tile_shape", "mf_sample_spectrum",
           "mf_sample_moments", "mf_shear_wiener", "mf_shear_sample", "mf_band_loss", "mf_sample_noalloc",
           "mf_plan_row_shape",
           "mf_plan_narrow_shape",
           "mf_status_string",
           "mf_last_error"]

_lib = None


def lib():
    """Load libmf.so (built by __graft_entry__.build()); fails loudly if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libmf.so not found at {LIB_PATH}: build it first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    # torch first: libmf's HIP runtime dependency must resolve to the runtime
    # torch already loaded, so that torch's device memory, streams and events
    # and the library's launches share one runtime.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.mf_plan_create.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(_Problem), C.c_uint32, vp]
    L.mf_plan_destroy.argtypes = [vp]
    L.mf_plan_set_spectrum.argtypes = [vp, C.c_int32, C.POINTER(_Spectrum), vp]
    L.mf_plan_reserve.argtypes = [vp, C.POINTER(_Reserve)]
    L.mf_band_loss.argtypes = [vp, vp, vp, vp, C.POINTER(_Schedule), vp, vp, vp, C.POINTER(Info), vp]
    L.mf_plan_pixel_offset.argtypes = [vp, C.c_int32]
    L.mf_plan_pixel_offset.restype = C.c_int64
    L.mf_plan_tau.argtypes = [vp, C.c_int32]
    L.mf_plan_tau.restype = C.c_double
    L.mf_plan_total_bands.argtypes = [vp]
    L.mf_plan_total_bands.restype = C.c_int32
    L.mf_wiener.argtypes = [vp, vp, C.POINTER(_Schedule), vp, vp, C.POINTER(Info), vp]
    L.mf_sample.argtypes = [vp, vp, C.POINTER(_SampleArgs), vp, vp, vp, vp]
    L.mf_sample_noalloc.argtypes = [vp, vp, C.POINTER(_SampleArgs), vp, vp, vp, vp]
    L.mf_wiener_backward.argtypes = [vp, vp, vp, C.POINTER(_Schedule), vp, vp, vp, C.POINTER(Info), vp]
    L.mf_band_power.argtypes = [vp, vp, vp, vp, vp]
    L.mf_wiener_backward_unrolled.argtypes = [vp, vp, C.POINTER(_Schedule), C.c_int32, vp, vp, vp, vp, vp]
    L.mf_plan_tile_shape.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.mf_plan_row_shape.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
    L.mf_plan_narrow_shape.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32)]
    L.mf_sample_spectrum.argtypes = [vp, vp, C.POINTER(_SpectrumArgs), vp, vp, vp, vp, vp, vp, vp]
    L.mf_sample_moments.argtypes = [vp, vp, C.c_int32, C.c_int32, vp, vp, vp]
    L.mf_shear_wiener.argtypes = [vp, vp, C.POINTER(_Schedule), C.c_float, vp, vp]
    L.mf_shear_sample.argtypes = [vp, vp, C.POINTER(_ShearArgs), vp, vp, vp, vp]
    L.mf_status_string.argtypes = [C.c_int]
    L.mf_status_string.restype = C.c_char_p
    L.mf_last_error.restype = C.c_char_p
    for name in ("mf_plan_create", "mf_plan_destroy", "mf_plan_reserve", "mf_band_loss", "mf_plan_set_spectrum",
                 "mf_wiener",
                 "mf_sample", "mf_sample_noalloc", "mf_wiener_backward", "mf_wiener_backward_unrolled",
                 "mf_band_power",
                 "mf_plan_tile_shape", "mf_plan_row_shape", "mf_plan_narrow_shape", "mf_sample_spectrum",
                 "mf_sample_moments",
                 "mf_shear_wiener",
                 "mf_shear_sample"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(status: int, allow_not_converged: bool = False):
    if status == MF_OK:
        return
    msg = lib().mf_last_error().decode()
    if status == MF_ERR_NOT_CONVERGED:
        if allow_not_converged:
            return
        raise NotConverged(status, msg)
    raise MFError(status, msg)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Schedule:
    """Cooling schedule: sweeps[j] sweeps at lambda[j], then (tol > 0) run the
    last level until the residual is <= tol, testing every check_every sweeps."""

    def __init__(self, lambdas: Sequence[float] = (1.0,), sweeps: Sequence[int] = (0,),
                 tol: float = 0.0, max_sweeps: int = 0, check_every: int = 10):
        self.lambdas = [float(x) for x in lambdas]
        self.sweeps = [int(x) for x in sweeps]
        self.tol, self.max_sweeps, self.check_every = float(tol), int(max_sweeps), int(check_every)

    @staticmethod
    def geometric(lam_start, lam_end, levels, sweeps_per_level, tol=0.0, max_sweeps=0, check_every=10):
        lams = list(np.geomspace(lam_start, lam_end, levels)) if levels > 1 else [lam_end]
        return Schedule(lams, [sweeps_per_level] * levels, tol, max_sweeps, check_every)

    @staticmethod
    def fixed(n_sweeps: int, lam: float = 1.0):
        return Schedule([lam], [n_sweeps])

    def _c(self):
        lam = (C.c_double * len(self.lambdas))(*self.lambdas)
        sw = (C.c_int32 * len(self.sweeps))(*self.sweeps)
        s = _Schedule(len(self.lambdas), lam, sw, self.tol, self.max_sweeps, self.check_every)
        s._keep = (lam, sw)
        return s


def _spectrum_c(spec):
    kind = getattr(spec, "kind")
    if kind == "powerlaw":
        return _Spectrum(MF_PK_POWERLAW, float(spec.amp), float(spec.k0), float(spec.n), 0, None, None), ()
    edges = np.ascontiguousarray(spec.edges, dtype=np.float64)
    amps = np.ascontiguousarray(spec.amps, dtype=np.float64)
    s = _Spectrum(MF_PK_BANDS, 0.0, 0.0, 0.0, len(amps),
                  edges.ctypes.data_as(C.POINTER(C.c_double)), amps.ctypes.data_as(C.POINTER(C.c_double)))
    return s, (edges, amps)


class Plan:
    """A set of image problems (size, noise variance map with +inf on missing
    pixels, isotropic power spectrum) with their device tables."""

    def __init__(self, problems, autotune: bool = False, graph: bool = False, streamed_solve: bool = False,
                 inf_as_1e8: bool = False):
        L = lib()
        self.problems = list(problems)
        keep = []
        arr = (_Problem * len(self.problems))()
        for i, p in enumerate(self.problems):
            nv = np.ascontiguousarray(p.noise_var, dtype=np.float32)
            spec, k = _spectrum_c(p.spectrum)
            keep += [nv, k]
            resp = getattr(p, "response", None)
            rp = None
            if resp is not None:
                r = np.ascontiguousarray(resp, dtype=np.float32)
                keep.append(r)
                rp = r.ctypes.data_as(C.POINTER(C.c_float))
            arr[i] = _Problem(int(p.H), int(p.W), nv.ctypes.data_as(C.POINTER(C.c_float)), spec, rp)
        h = C.c_void_p()
        flags = ((MF_FLAG_AUTOTUNE if autotune else 0) | (MF_FLAG_GRAPH if graph else 0)
                 | (MF_FLAG_STREAMED_SOLVE if streamed_solve else 0) | (MF_FLAG_INF_AS_1E8 if inf_as_1e8 else 0))
        _check(L.mf_plan_create(C.byref(h), len(self.problems), arr, flags, None))
        self._h = h
        self.offsets = [L.mf_plan_pixel_offset(h, i) for i in range(len(self.problems) + 1)]
        self.total_pixels = self.offsets[-1]
        self.total_bands = L.mf_plan_total_bands(h)

    def close(self):
        if getattr(self, "_h", None):
            lib().mf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tau(self, i: int) -> float:
        return lib().mf_plan_tau(self._h, i)

    def set_spectrum(self, i: int, spectrum):
        s, keep = _spectrum_c(spectrum)
        _check(lib().mf_plan_set_spectrum(self._h, i, C.byref(s), _stream()))

    def reserve(self, calls, chains: int = 1, storage: str = "fp32", unrolled_sweeps: int = 0,
                checkpoint_every: int = 0):
        """Allocate the workspaces of the named calls ("solve", "sample",
        "spectrum", "shear", "unrolled", "moments") now, so that those calls
        allocate nothing (and can be captured into a graph)."""
        bits = 0
        for c in ([calls] if isinstance(calls, str) else calls):
            bits |= RESERVE[c]
        r = _Reserve(bits, int(chains), STORAGES[storage], int(unrolled_sweeps), int(checkpoint_every))
        _check(lib().mf_plan_reserve(self._h, C.byref(r)))

    def set_band_amplitudes(self, theta):
        """Replace the band amplitudes of every band-spectrum problem;
        `theta` concatenates them in problem order (length total_bands)."""
        import types
        theta = np.asarray(theta, dtype=np.float64)
        if theta.shape != (self.total_bands,):
            raise ValueError(f"need {self.total_bands} band amplitudes")
        o = 0
        for i, p in enumerate(self.problems):
            if getattr(p.spectrum, "kind", None) != "bands":
                continue
            nb = len(p.spectrum.amps)
            spec = types.SimpleNamespace(kind="bands", edges=p.spectrum.edges, amps=theta[o:o + nb])
            self.set_spectrum(i, spec)
            o += nb

    # ---- data marshalling helpers (host numpy <-> concatenated device arrays)
    def concat(self, arrays, device="cuda"):
        import torch
        flat = np.concatenate([np.asarray(a, dtype=np.float32).ravel() for a in arrays])
        return torch.from_numpy(flat).to(device)

    def split(self, flat):
        x = flat.detach().cpu().numpy()
        return [x[self.offsets[i]:self.offsets[i + 1]].reshape(p.H, p.W)
                for i, p in enumerate(self.problems)]

    # ---- entry points
    def wiener(self, d, schedule: Schedule, s_init=None, out=None, allow_not_converged=False, want_info=True):
        """Wiener filter (concatenated).  want_info=False passes no info array,
        so that a fixed schedule neither synchronises nor copies to the host
        (the call can then be captured into a graph); the info list is empty."""
        import torch
        out = torch.empty_like(d) if out is None else out
        info = (Info * len(self.problems))() if want_info else None
        sch = schedule._c()
        st = lib().mf_wiener(self._h, _ptr(d), C.byref(sch), _ptr(s_init), _ptr(out), info, _stream())
        _check(st, allow_not_converged)
        return out, (list(info) if want_info else [])

    def samples_buffer(self, chains: int, n_samples: int, device="cuda"):
        import torch
        return torch.empty(chains * n_samples * self.total_pixels, dtype=torch.float32, device=device)

    def sample(self, d, seed: int, chains: int, burn_in: int, n_samples: int, thin: int = 1,
               sweep_offset: int = 0, init_scale: float = 0.0, form: str = "auto",
               state_in=None, state_out=None, samples=True, out=None, storage: str = "fp32",
               cooling: Optional["Schedule"] = None, check_finite: bool = True):
        """Returns (samples [concat over problems of chains*n_samples*H*W] or None,
        state_out or None).  `out` may hold a preallocated samples buffer.
        `storage` ("fp32", "fp16", "bf16") is the precision of the streamed
        field between kernels (streamed and plain forms).  `cooling` levels
        (lambda >= 1, sweeps) run before the burn-in."""
        if out is None and samples and n_samples > 0:
            out = self.samples_buffer(chains, n_samples, d.device)
        if out is not None and out.numel() < chains * n_samples * self.total_pixels:
            raise ValueError("samples buffer too small")
        cool = cooling._c() if cooling is not None else None
        args = _SampleArgs(int(seed), int(chains), int(burn_in), int(n_samples), int(thin),
                           int(sweep_offset), float(init_scale), FORMS[form], STORAGES[storage],
                           int(bool(check_finite)), C.pointer(cool) if cool is not None else None)
        st = lib().mf_sample(self._h, _ptr(d), C.byref(args), _ptr(state_in), _ptr(state_out),
                             _ptr(out), _stream())
        _check(st)
        return out, state_out

    def sample_view(self, flat, problem: int, chains: int, n_samples: int):
        p = self.problems[problem]
        off = chains * n_samples * self.offsets[problem]
        return flat[off:off + chains * n_samples * p.H * p.W].view(chains, n_samples, p.H, p.W)

    def state_buffer(self, chains: int, device="cuda"):
        import torch
        pairs = (chains + 1) // 2
        return torch.zeros(2 * pairs * self.total_pixels, dtype=torch.float32, device=device)

    @property
    def band_offsets(self):
        """First band of each problem in concatenated band arrays (plan order)."""
        out, o = [], 0
        for p in self.problems:
            out.append(o)
            if p.spectrum.kind == "bands":
                o += len(p.spectrum.amps)
        return out + [o]

    def sample_spectrum(self, d, seed: int, chains: int, burn_in: int, n_samples: int, thin: int = 1,
                        sweeps_per_draw: int = 1, prior_dof: int = 0, prior_beta: float = 0.0,
                        iteration_offset: int = 0, init_scale: float = 0.0, state_in=None, theta_in=None,
                        state_out=None, theta_out=None, samples=False, theta_samples=True,
                        check_finite: bool = True):
        """Hierarchical sampler (signal and band amplitudes).  Returns
        (theta samples [concat over problems of chains*n_samples*bands] float64 or
        None, signal samples or None, state_out, theta_out)."""
        import torch
        dev = d.device
        pairs = (chains + 1) // 2
        if theta_out is None:
            theta_out = torch.empty(2 * pairs * self.total_bands, dtype=torch.float64, device=dev)
        ts = None
        if theta_samples and n_samples > 0:
            ts = torch.empty(chains * n_samples * self.total_bands, dtype=torch.float64, device=dev)
        smp = self.samples_buffer(chains, n_samples, dev) if samples and n_samples > 0 else None
        args = _SpectrumArgs(int(seed), int(chains), int(burn_in), int(n_samples), int(thin),
                             int(sweeps_per_draw), int(prior_dof), float(prior_beta), int(iteration_offset),
                             float(init_scale), int(bool(check_finite)))
        _check(lib().mf_sample_spectrum(self._h, _ptr(d), C.byref(args), _ptr(state_in), _ptr(theta_in),
                                        _ptr(state_out), _ptr(theta_out), _ptr(smp), _ptr(ts), _stream()))
        return ts, smp, state_out, theta_out

    # ---- mass mapping (complex shear data, spin-2 operator)
    def concat_complex(self, arrays, device="cuda"):
        """Concatenate complex images into one complex64 device tensor."""
        import torch
        flat = np.concatenate([np.asarray(a, dtype=np.complex64).ravel() for a in arrays])
        return torch.from_numpy(flat).to(device)

    def split_complex(self, flat):
        x = flat.detach().cpu().numpy()
        return [x[self.offsets[i]:self.offsets[i + 1]].reshape(p.H, p.W) for i, p in enumerate(self.problems)]

    def shear_wiener(self, gamma, schedule: Schedule, b_ratio: float = 0.0, out=None):
        """Convergence Wiener filter (complex, concatenated) of complex shear data."""
        import torch
        out = torch.empty_like(gamma) if out is None else out
        sch = schedule._c()
        _check(lib().mf_shear_wiener(self._h, _ptr(gamma), C.byref(sch), float(b_ratio), _ptr(out), _stream()))
        return out

    def shear_state_buffer(self, chains: int, device="cuda"):
        import torch
        return torch.zeros(chains * self.total_pixels, dtype=torch.complex64, device=device)

    def shear_sample(self, gamma, seed: int, chains: int, burn_in: int, n_samples: int, thin: int = 1,
                     sweep_offset: int = 0, b_ratio: float = 0.0, state_in=None, state_out=None, samples=True,
                     check_finite: bool = True):
        """Samples of the convergence, complex [concat over problems of chains*n_samples*H*W]."""
        import torch
        out = None
        if samples and n_samples > 0:
            out = torch.empty(chains * n_samples * self.total_pixels, dtype=torch.complex64, device=gamma.device)
        args = _ShearArgs(int(seed), int(chains), int(burn_in), int(n_samples), int(thin), int(sweep_offset),
                          float(b_ratio), int(bool(check_finite)))
        _check(lib().mf_shear_sample(self._h, _ptr(gamma), C.byref(args), _ptr(state_in), _ptr(state_out),
                                     _ptr(out), _stream()))
        return out, state_out

    def sample_moments(self, samples, chains: int, n_samples: int, want_var: bool = True):
        """Per-pixel (mean, variance) over chains and samples, float64, concatenated."""
        import torch
        mean = torch.empty(self.total_pixels, dtype=torch.float64, device=samples.device)
        var = torch.empty_like(mean) if want_var else None
        _check(lib().mf_sample_moments(self._h, _ptr(samples), int(chains), int(n_samples), _ptr(mean), _ptr(var),
                                       _stream()))
        return mean, var

    def theta_view(self, flat, problem: int, chains: int, n_samples: int):
        """Band-amplitude samples [chains, n_samples, bands] of one problem."""
        b0, b1 = self.band_offsets[problem], self.band_offsets[problem + 1]
        nb = b1 - b0
        off = chains * n_samples * b0
        return flat[off:off + chains * n_samples * nb].view(chains, n_samples, nb)

    def tile_shape(self, H: int, W: int):
        """(columns, threads) of the column-kernel tile used for size class H x W."""
        c, t = C.c_int32(), C.c_int32()
        _check(lib().mf_plan_tile_shape(self._h, int(H), int(W), C.byref(c), C.byref(t)))
        return c.value, t.value

    def row_shape(self, H: int, W: int) -> int:
        """Rows per workgroup of the fused row kernel for size class H x W (0: none)."""
        r = C.c_int32()
        _check(lib().mf_plan_row_shape(self._h, int(H), int(W), C.byref(r)))
        return r.value

    def narrow_shape(self, H: int, W: int):
        """(columns, threads, rows) used for size class H x W by launches too small to fill the GPU."""
        c, t, r = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().mf_plan_narrow_shape(self._h, int(H), int(W), C.byref(c), C.byref(t), C.byref(r)))
        return c.value, t.value, r.value

    def state_view(self, flat, problem: int, chains: int):
        """Complex pair states [pairs, H, W] of one problem in a state buffer."""
        import torch
        p = self.problems[problem]
        pairs = (chains + 1) // 2
        off = 2 * pairs * self.offsets[problem]
        return torch.view_as_complex(flat[off:off + 2 * pairs * p.H * p.W].view(pairs, p.H, p.W, 2))

    def wiener_backward(self, s_wf, grad_s, schedule: Schedule, want_bands=True, want_v=False,
                        allow_not_converged=False):
        import torch
        grad_d = torch.empty_like(grad_s)
        gb = None
        if want_bands and self.total_bands > 0:
            gb = torch.zeros(self.total_bands, dtype=torch.float64, device=grad_s.device)
        v = torch.empty_like(grad_s) if want_v else None
        info = (Info * len(self.problems))()
        sch = schedule._c()
        st = lib().mf_wiener_backward(self._h, _ptr(s_wf), _ptr(grad_s), C.byref(sch), _ptr(grad_d),
                                      _ptr(gb), _ptr(v), info, _stream())
        _check(st, allow_not_converged)
        return grad_d, gb, v, list(info)

    def wiener_backward_unrolled(self, d, grad_s, schedule: Schedule, checkpoint_every: int = 20,
                                 want_bands=True):
        """Gradient of the truncated iteration: returns (s_K, grad_d, grad_bands)."""
        import torch
        s_out = torch.empty_like(grad_s)
        grad_d = torch.empty_like(grad_s)
        gb = None
        if want_bands and self.total_bands > 0:
            gb = torch.zeros(self.total_bands, dtype=torch.float64, device=grad_s.device)
        sch = schedule._c()
        _check(lib().mf_wiener_backward_unrolled(self._h, _ptr(d), C.byref(sch), int(checkpoint_every),
                                                 _ptr(grad_s), _ptr(s_out), _ptr(grad_d), _ptr(gb), _stream()))
        return s_out, grad_d, gb

    def band_loss(self, d, s_wf, s_true, adjoint_schedule: Optional[Schedule] = None, want_grad=True,
                  allow_not_converged=False):
        """Loss of the differentiation workload at the Wiener filter s_wf
        (mf_band_loss): returns (loss per problem float64, grad_d or None,
        grad_bands or None, adjoint info)."""
        import torch
        loss = torch.empty(len(self.problems), dtype=torch.float64, device=d.device)
        gd = torch.empty_like(d) if want_grad else None
        gb = torch.zeros(max(self.total_bands, 1), dtype=torch.float64, device=d.device) if want_grad else None
        info = (Info * len(self.problems))()
        sch = adjoint_schedule._c() if adjoint_schedule is not None else None
        st = lib().mf_band_loss(self._h, _ptr(d), _ptr(s_wf), _ptr(s_true), C.byref(sch) if sch is not None else None,
                                _ptr(loss), _ptr(gd), _ptr(gb), info, _stream())
        _check(st, allow_not_converged)
        return loss, gd, (gb[:self.total_bands] if gb is not None else None), list(info)

    def band_power(self, x, y):
        import torch
        out = torch.zeros(max(self.total_bands, 1), dtype=torch.float64, device=x.device)
        _check(lib().mf_band_power(self._h, _ptr(x), _ptr(y), _ptr(out), _stream()))
        return out[:self.total_bands]
