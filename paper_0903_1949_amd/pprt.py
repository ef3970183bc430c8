"""Thin Python binding of libpprt (C ABI in include/pprt.h).

Argument marshalling only: every step of the formal solution, the profile
quadratures and the ALI update runs in the library's HIP kernels.  PyTorch
supplies device memory and the stream; no torch type crosses the ABI.  The
binding refuses to run without the compiled library -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpprt.so")

FP64, FP32 = 0, 1
BC_DIFFUSION, BC_GIVEN = 0, 1
THICK_RULE, THICK_NEVER, THICK_ALWAYS = 0, 1, 2
OUT_J, OUT_JMS, OUT_LSTAR, OUT_LSTAR_C = 0x01, 0x02, 0x04, 0x08
OUT_IPLUS, OUT_IMINUS, OUT_H, OUT_IEMERG = 0x10, 0x20, 0x40, 0x80
OUT_LSTAR_SUB, OUT_LSTAR_SUP = 0x100, 0x200
OUT_ALL = 0xFF
OUTPUT_NAMES = {OUT_J: "J", OUT_JMS: "JmS", OUT_LSTAR: "lstar", OUT_LSTAR_C: "lstar_c",
                OUT_IPLUS: "Iplus", OUT_IMINUS: "Iminus", OUT_H: "H", OUT_IEMERG: "Iemerg",
                OUT_LSTAR_SUB: "lstar_sub", OUT_LSTAR_SUP: "lstar_sup"}
LSTAR_DIAG, LSTAR_TRI = 0, 1

STATUS = {0: "OK", 1: "E_INVALID_ARG", 2: "E_SHAPE", 3: "E_DEVICE", 4: "E_WORKSPACE",
          5: "E_NONFINITE", 6: "E_NOT_CONVERGED", 7: "E_SINGULAR", 8: "E_UNSUPPORTED",
          9: "E_LAUNCH"}


class VoxGrid(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nt", C.c_int32), ("np", C.c_int32), ("r", C.POINTER(C.c_double))]


class VoxInfo(C.Structure):
    _fields_ = [("nvox", C.c_int64), ("ndir", C.c_int64), ("nrays", C.c_int64), ("nsegments", C.c_int64),
                ("ncoverage", C.c_int64), ("spacing", C.c_double), ("device_bytes", C.c_size_t)]


class PprtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class Shape(C.Structure):
    _fields_ = [("nbatch", C.c_int32), ("nd", C.POINTER(C.c_int32)), ("na", C.c_int32),
                ("nf", C.c_int32), ("precision", C.c_int32), ("lower_bc", C.c_int32),
                ("outputs", C.c_uint32), ("waves_per_block", C.c_int32)]


class FsIn(C.Structure):
    _fields_ = [("tau", C.c_void_p), ("q", C.c_void_p), ("Sg", C.c_void_p), ("Itop", C.c_void_p),
                ("Bbot", C.c_void_p), ("Bbot_prev", C.c_void_p), ("Ibot", C.c_void_p)]


class FsOut(C.Structure):
    _fields_ = [("J", C.c_void_p), ("JmS", C.c_void_p), ("lstar", C.c_void_p),
                ("lstar_c", C.c_void_p), ("Iplus", C.c_void_p), ("Iminus", C.c_void_p),
                ("H", C.c_void_p), ("Iemerg", C.c_void_p), ("lstar_sub", C.c_void_p),
                ("lstar_sup", C.c_void_p)]


class FsGrad(C.Structure):
    _fields_ = [("dq", C.c_void_p), ("dSg", C.c_void_p), ("dBbot", C.c_void_p),
                ("dBbot_prev", C.c_void_p), ("dIbot", C.c_void_p)]


class TuneReport(C.Structure):
    _fields_ = [("waves_per_block", C.c_int32), ("persistent_waves_per_cu", C.c_int32),
                ("best_ms", C.c_float), ("default_ms", C.c_float), ("candidates", C.c_int32),
                ("from_cache", C.c_int32)]


class Peaks(C.Structure):
    _fields_ = [("fp32_tflops", C.c_double), ("fp64_tflops", C.c_double),
                ("exp2_trate", C.c_double), ("copy_gbs", C.c_double),
                ("atomic_f64_gadds", C.c_double), ("atomic_f32_gadds", C.c_double)]


class TwoLevel(C.Structure):
    _fields_ = [("eps", C.c_void_p), ("B", C.c_void_p), ("wphi", C.c_void_p)]


class Continuum(C.Structure):
    _fields_ = [("pfrac", C.c_void_p), ("sg_const", C.c_void_p), ("omega", C.c_void_p)]


class Atom(C.Structure):
    _fields_ = [("nlev", C.c_int32), ("ntr", C.c_int32)] + [
        (n, C.c_void_p) for n in ("lower", "upper", "k0", "k1", "owner", "sigma", "bfac", "W", "G",
                                  "Bnu", "kc", "sc", "ntot", "Cul", "Clu", "nu", "line_nu0",
                                  "line_s", "line_a", "dopp")]


class AliCtl(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("iters_per_sync", C.c_int32),
                ("use_graph", C.c_int32), ("resume", C.c_int32)]


class AliReport(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("n_converged", C.c_int32), ("max_rel", C.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpprt.so (built in-tree by paper_0903_1949_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpprt.so not found at {path}: build it first "
                           "(python -m paper_0903_1949_amd.build); there is no CPU fallback")
    lib = C.CDLL(path)
    P, I, D, U32 = C.c_void_p, C.c_int, C.c_double, C.c_uint32
    sig = {
        "pprt_version": (I, [C.POINTER(I), C.POINTER(I), C.POINTER(I)]),
        "pprt_status_string": (C.c_char_p, [I]),
        "pprt_gauss_legendre01": (I, [I, C.POINTER(D), C.POINTER(D)]),
        "pprt_create": (I, [C.POINTER(P), I]),
        "pprt_destroy": (None, [P]),
        "pprt_set_stream": (I, [P, P]),
        "pprt_last_error": (C.c_char_p, [P]),
        "pprt_sync": (I, [P, C.POINTER(U32)]),
        "pprt_shape_check": (I, [C.POINTER(Shape), C.c_char_p, C.c_size_t]),
        "pprt_plan_create": (I, [P, C.POINTER(Shape), C.POINTER(D), C.POINTER(D), C.POINTER(P)]),
        "pprt_plan_destroy": (None, [P]),
        "pprt_plan_workspace_bytes": (I, [P, C.POINTER(C.c_size_t)]),
        "pprt_plan_info": (I, [P, C.POINTER(C.c_int64), C.POINTER(D), C.POINTER(D)]),
        "pprt_formal_solution": (I, [P, C.POINTER(FsIn), C.POINTER(FsOut)]),
        "pprt_two_level_ali_step": (I, [P, C.POINTER(FsIn), C.POINTER(TwoLevel), P, P, P, P]),
        "pprt_plan_scattering_workspace_bytes": (I, [P, C.POINTER(C.c_size_t)]),
        "pprt_formal_solution_scattering": (I, [P, C.POINTER(FsIn), P, C.POINTER(FsOut), P]),
        "pprt_plan_set_thick_mode": (I, [P, C.c_int32]),
        "pprt_thick_counts": (I, [P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
        "pprt_thick_counts_reset": (I, [P]),
        "pprt_plan_continuum_workspace_bytes": (I, [P, C.POINTER(C.c_size_t)]),
        "pprt_two_level_ali_step_continuum": (I, [P, C.POINTER(FsIn), C.POINTER(TwoLevel),
                                                  C.POINTER(Continuum), P, P, P, P]),
        "pprt_atom_check": (I, [P, C.POINTER(Atom)]),
        "pprt_nlte_opacity": (I, [P, C.POINTER(Atom), P, P, P, P]),
        "pprt_rates_assemble": (I, [P, C.POINTER(Atom), P, P, P, P, P, P]),
        "pprt_rates_solve": (I, [P, C.POINTER(Atom), P, P, P, P, P, P]),
        "pprt_plan_nlte_workspace_bytes": (I, [P, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
        "pprt_nlte_step": (I, [P, C.POINTER(FsIn), C.POINTER(Atom), P, P, P]),
        "pprt_two_level_moments": (I, [P, C.POINTER(FsIn), C.POINTER(TwoLevel), P, P, P]),
        "pprt_two_level_update": (I, [P, C.POINTER(TwoLevel), P, P, P, P]),
        "pprt_two_level_ali": (I, [P, C.POINTER(FsIn), C.POINTER(TwoLevel), C.POINTER(AliCtl),
                                   P, P, C.POINTER(AliReport), P]),
        "pprt_plan_adjoint_workspace_bytes": (I, [P, C.c_int32, C.POINTER(C.c_size_t)]),
        "pprt_plan_set_launch": (I, [P, C.c_int32, C.c_int32]),
        "pprt_measure_peaks": (I, [P, P, C.c_size_t, C.POINTER(Peaks)]),
        "pprt_voigt": (I, [P, C.c_int64, P, P, P]),
        "pprt_plan_set_operator": (I, [P, C.c_int32, C.c_int32]),
        "pprt_two_level_reset": (I, [P, P]),
        "pprt_plan_get_launch": (I, [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "pprt_plan_autotune": (I, [P, C.POINTER(FsIn), C.POINTER(TwoLevel), P, P, C.c_int32,
                                   C.POINTER(TuneReport)]),
        "pprt_emergent_intensity": (I, [P, C.POINTER(FsIn), C.c_int32, P, P]),
        "pprt_formal_solution_vjp": (I, [P, C.POINTER(FsIn), C.c_int32, P, C.POINTER(FsGrad), P]),
        "pprt_plan_scattering_vjp_workspace_bytes": (I, [P, C.POINTER(C.c_size_t)]),
        "pprt_formal_solution_scattering_vjp": (I, [P, C.POINTER(FsIn), P, P, C.POINTER(FsGrad), P]),
        "pprt_vox_plan_create": (I, [P, C.POINTER(VoxGrid), C.c_int32, C.c_int32, D, C.c_int32, C.c_int32,
                                     C.POINTER(P)]),
        "pprt_vox_plan_info": (I, [P, C.POINTER(VoxInfo)]),
        "pprt_vox_directions": (I, [P, C.POINTER(D), C.POINTER(D)]),
        "pprt_vox_plan_destroy": (None, [P]),
        "pprt_vox_geometry_host": (I, [C.POINTER(VoxGrid), C.c_int32, C.c_int32, D, C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int64), P, P, P, P, P, P]),
        "pprt_vox_formal_solution": (I, [P, P, P, P, P, P, P, P]),
        "pprt_vox_ali_workspace_bytes": (I, [P, C.POINTER(C.c_size_t)]),
        "pprt_vox_ali_step": (I, [P, P, P, P, P, P, P, P, P]),
        "pprt_sph_plan_create": (I, [P, C.c_int32, C.POINTER(C.c_int32), C.c_int32, C.c_int32,
                                     C.c_int32, U32, C.POINTER(D), C.c_int32, C.POINTER(P)]),
        "pprt_sph_plan_destroy": (None, [P]),
        "pprt_sph_plan_info": (I, [P, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int64)]),
        "pprt_sph_formal_solution": (I, [P, C.POINTER(FsIn), C.POINTER(FsOut)]),
        "pprt_sph_plan_workspace_bytes": (I, [P, C.POINTER(C.c_size_t)]),
        "pprt_sph_two_level_ali_step": (I, [P, C.POINTER(FsIn), C.POINTER(TwoLevel), P, P, P, P]),
        "pprt_sph_two_level_moments": (I, [P, C.POINTER(FsIn), C.POINTER(TwoLevel), P, P, P]),
        "pprt_sph_two_level_update": (I, [P, C.POINTER(TwoLevel), P, P, P, P]),
        "pprt_set_validation": (I, [P, U32]),
        "pprt_check_tau": (I, [C.c_int32, C.POINTER(C.c_int32), C.POINTER(D), C.c_char_p, C.c_size_t]),
        "pprt_check_finite": (I, [C.c_int32, C.c_int64, P, C.c_char_p, C.c_size_t]),
        "pprt_atom_check_host": (I, [C.POINTER(Atom), C.c_int64, C.c_int32, C.c_char_p, C.c_size_t]),
        "pprt_nlte_solve": (I, [P, C.POINTER(FsIn), C.POINTER(Atom), C.POINTER(AliCtl), P, P,
                                C.POINTER(AliReport), P]),
        "pprt_two_level_ali_step_noalloc": (I, [P, C.POINTER(FsIn), C.POINTER(TwoLevel), P, P, P]),
        "pprt_two_level_graph_create": (I, [P, C.POINTER(FsIn), C.POINTER(TwoLevel), P, P, P, P,
                                            C.c_int32, C.POINTER(P)]),
        "pprt_graph_launch": (I, [P]),
        "pprt_graph_destroy": (None, [P]),
        "pprt_ali_state_bytes": (I, [P, C.POINTER(C.c_size_t)]),
        "pprt_ali_state_export": (I, [P, P, P, P, C.c_size_t]),
        "pprt_ali_state_import": (I, [P, P, C.c_size_t, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def declared_symbols(header: str | None = None):
    """Function names declared in include/pprt.h (used by the ABI test)."""
    import re
    header = header or os.path.join(os.path.dirname(HERE), "include", "pprt.h")
    text = open(header).read()
    return sorted(set(re.findall(r"\b(pprt_[a-z0-9_]+)\s*\(", text)))


def gauss_legendre01(n: int):
    lib = load_library()
    mu = np.zeros(n)
    w = np.zeros(n)
    st = lib.pprt_gauss_legendre01(n, mu.ctypes.data_as(C.POINTER(C.c_double)),
                                   w.ctypes.data_as(C.POINTER(C.c_double)))
    if st != 0:
        raise PprtError(st, "gauss_legendre01")
    return mu, w


def shape_check(nd, na, nf, precision=FP32, lower_bc=BC_DIFFUSION, outputs=OUT_JMS,
                waves_per_block=0):
    """Host-only shape validation (pprt_shape_check): (status name, message)."""
    lib = load_library()
    ndv = np.ascontiguousarray(np.asarray(nd, dtype=np.int32))
    sh = Shape(int(ndv.shape[0]), ndv.ctypes.data_as(C.POINTER(C.c_int32)) if ndv.size else None,
               int(na), int(nf), int(precision), int(lower_bc), int(outputs), int(waves_per_block))
    buf = C.create_string_buffer(256)
    st = lib.pprt_shape_check(C.byref(sh), buf, 256)
    return STATUS.get(st, st), buf.value.decode()


def check_tau(nd, tau):
    """Host-only pprt_check_tau: (status name, message)."""
    lib = load_library()
    ndv = np.ascontiguousarray(np.asarray(nd, dtype=np.int32))
    tv = np.ascontiguousarray(np.asarray(tau, dtype=np.float64))
    buf = C.create_string_buffer(256)
    st = lib.pprt_check_tau(int(ndv.shape[0]), ndv.ctypes.data_as(C.POINTER(C.c_int32)),
                            tv.ctypes.data_as(C.POINTER(C.c_double)), buf, 256)
    return STATUS.get(st, st), buf.value.decode()


def check_finite(x):
    """Host-only pprt_check_finite on a float32 or float64 numpy array."""
    lib = load_library()
    x = np.ascontiguousarray(x)
    if x.dtype not in (np.float32, np.float64):
        raise TypeError("float32 or float64 array expected")
    buf = C.create_string_buffer(256)
    st = lib.pprt_check_finite(FP64 if x.dtype == np.float64 else FP32, int(x.size),
                               C.c_void_p(x.ctypes.data), buf, 256)
    return STATUS.get(st, st), buf.value.decode()


def atom_check_host(atom, rows=None):
    """Host-only pprt_atom_check_host on a workloads.MultiLevelAtom (its
    index tables, cross-sections and collision rates): (status, message)."""
    lib = load_library()
    keep = {"lower": np.ascontiguousarray(atom.lo, dtype=np.int32),
            "upper": np.ascontiguousarray(atom.up, dtype=np.int32),
            "k0": np.ascontiguousarray(atom.k0, dtype=np.int32),
            "k1": np.ascontiguousarray(atom.k1, dtype=np.int32),
            "owner": np.ascontiguousarray(atom.owner, dtype=np.int32),
            "sigma": np.ascontiguousarray(atom.sigma, dtype=np.float64),
            "Cul": np.ascontiguousarray(atom.Cul, dtype=np.float64),
            "Clu": np.ascontiguousarray(atom.Clu, dtype=np.float64)}
    if getattr(atom, "line_a", None) is not None:
        keep.update(line_nu0=np.ascontiguousarray(atom.line_nu0, dtype=np.float64),
                    line_s=np.ascontiguousarray(atom.line_s, dtype=np.float64),
                    line_a=np.ascontiguousarray(atom.line_a, dtype=np.float64))
    a = Atom(int(atom.nl), int(atom.nt), **{k: C.c_void_p(v.ctypes.data) for k, v in keep.items()})
    rows = int(keep["Cul"].shape[0]) if rows is None else int(rows)
    buf = C.create_string_buffer(256)
    st = lib.pprt_atom_check_host(C.byref(a), rows, int(keep["owner"].shape[0]), buf, 256)
    return STATUS.get(st, st), buf.value.decode()


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """A libpprt context on one HIP device, enqueueing on torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load_library()
        self.device = device
        h = C.c_void_p()
        st = self.lib.pprt_create(C.byref(h), device)
        if st != 0:
            raise PprtError(st, f"pprt_create(device={device})")
        self.h = h
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.set_stream(stream)

    def set_stream(self, stream):
        self.stream = stream
        self._check(self.lib.pprt_set_stream(self.h, C.c_void_p(stream.cuda_stream)), "set_stream")

    def _check(self, st, what):
        if st != 0:
            msg = self.lib.pprt_last_error(self.h)
            raise PprtError(st, f"{what}: {msg.decode() if msg else ''}")

    def sync(self) -> int:
        s = C.c_uint32(0)
        self._check(self.lib.pprt_sync(self.h, C.byref(s)), "sync")
        return s.value

    def set_validation(self, on: bool = True):
        """pprt_set_validation: host scan of every input before each launch."""
        self._check(self.lib.pprt_set_validation(self.h, 1 if on else 0), "set_validation")

    def thick_counts(self, reset: bool = False) -> tuple[int, int]:
        """pprt_thick_counts: (eliminations run in FP64, all eliminations) of
        the FP32-bulk scattering path since creation or the last reset."""
        f64, tot = C.c_uint64(0), C.c_uint64(0)
        self._check(self.lib.pprt_thick_counts(self.h, C.byref(f64), C.byref(tot)), "thick_counts")
        if reset:
            self._check(self.lib.pprt_thick_counts_reset(self.h), "thick_counts_reset")
        return int(f64.value), int(tot.value)

    def voigt(self, a, x):
        """pprt_voigt: H(a, x) for device float64 tensors of equal length."""
        import torch
        a = a.contiguous(); x = x.contiguous()
        if a.dtype != torch.float64 or x.dtype != torch.float64 or a.shape != x.shape:
            raise TypeError("a and x must be float64 tensors of one shape")
        H = torch.empty_like(x)
        self._check(self.lib.pprt_voigt(self.h, x.numel(), _ptr(a), _ptr(x), _ptr(H)), "voigt")
        return H

    def measure_peaks(self, scratch_mib: int = 1024) -> dict:
        """pprt_measure_peaks with a scratch buffer of scratch_mib MiB."""
        import torch
        buf = torch.empty(scratch_mib << 20, dtype=torch.uint8, device=f"cuda:{self.device}")
        pk = Peaks()
        self._check(self.lib.pprt_measure_peaks(self.h, _ptr(buf), buf.numel(), C.byref(pk)),
                    "measure_peaks")
        return {k: getattr(pk, k) for k, _ in Peaks._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.pprt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Validated shape of a ragged batch of atmospheres (see pprt_plan_create)."""

    def __init__(self, ctx: Context, nd, na: int, nf: int, precision: int = FP32,
                 lower_bc: int = BC_DIFFUSION, outputs: int = OUT_JMS | OUT_LSTAR_C,
                 waves_per_block: int = 0, mu=None, w=None):
        import torch
        self.ctx = ctx
        self.lib = ctx.lib
        self.nd = np.ascontiguousarray(np.asarray(nd, dtype=np.int32))
        self.na, self.nf, self.precision = int(na), int(nf), int(precision)
        self.lower_bc, self.outputs = int(lower_bc), int(outputs)
        sh = Shape(int(self.nd.shape[0]), self.nd.ctypes.data_as(C.POINTER(C.c_int32)), self.na,
                   self.nf, self.precision, self.lower_bc, self.outputs, int(waves_per_block))
        h = C.c_void_p()
        if (mu is None) != (w is None):
            raise ValueError("give both mu and w or neither")
        mup = wp = None
        if mu is not None:
            self._mu = np.ascontiguousarray(mu, dtype=np.float64)
            self._w = np.ascontiguousarray(w, dtype=np.float64)
            mup = self._mu.ctypes.data_as(C.POINTER(C.c_double))
            wp = self._w.ctypes.data_as(C.POINTER(C.c_double))
        ctx._check(self.lib.pprt_plan_create(ctx.h, C.byref(sh), mup, wp, C.byref(h)), "plan_create")
        self.h = h
        rows = C.c_int64()
        self.mu = np.zeros(self.na)
        self.w = np.zeros(self.na)
        ctx._check(self.lib.pprt_plan_info(h, C.byref(rows), self.mu.ctypes.data_as(C.POINTER(C.c_double)),
                                           self.w.ctypes.data_as(C.POINTER(C.c_double))), "plan_info")
        self.rows = rows.value
        nb = C.c_size_t()
        ctx._check(self.lib.pprt_plan_workspace_bytes(h, C.byref(nb)), "workspace_bytes")
        self.workspace_bytes = nb.value
        self.dtype = torch.float64 if self.precision == FP64 else torch.float32
        self._ws = None

    @property
    def nb(self) -> int:
        return int(self.nd.shape[0])

    def workspace(self):
        import torch
        if self._ws is None:
            self._ws = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8,
                                   device=f"cuda:{self.ctx.device}")
        return self._ws

    def close(self):
        if getattr(self, "h", None):
            self.lib.pprt_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------- checks
    def _want(self, t, shape, dtype, name):
        import torch
        if t is None:
            raise ValueError(f"{name} is required")
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def fs_in(self, tau, q, Sg=None, Bbot=None, Bbot_prev=None, Itop=None, Ibot=None):
        import torch
        R, nf, na, nb, dt = self.rows, self.nf, self.na, self.nb, self.dtype
        self._want(tau, (R,), torch.float64, "tau")
        self._want(q, (R, nf), dt, "q")
        if Sg is not None:
            self._want(Sg, (R, nf), dt, "Sg")
        if Bbot is not None:
            self._want(Bbot, (nb, nf), dt, "Bbot")
        if Bbot_prev is not None:
            self._want(Bbot_prev, (nb, nf), dt, "Bbot_prev")
        if Itop is not None:
            self._want(Itop, (nb, nf, na), dt, "Itop")
        if Ibot is not None:
            self._want(Ibot, (nb, nf, na), dt, "Ibot")
        return FsIn(_ptr(tau), _ptr(q), _ptr(Sg), _ptr(Itop), _ptr(Bbot), _ptr(Bbot_prev), _ptr(Ibot))

    # ------------------------------------------------------- entry points
    def formal_solution(self, tau, q, Sg, Bbot=None, Bbot_prev=None, Itop=None, Ibot=None,
                        out: dict | None = None) -> dict:
        """pprt_formal_solution: returns a dict of the requested outputs."""
        import torch
        fin = self.fs_in(tau, q, Sg, Bbot, Bbot_prev, Itop, Ibot)
        R, nf, na, nb = self.rows, self.nf, self.na, self.nb
        shapes = {"J": (R, nf), "JmS": (R, nf), "lstar": (R, nf), "lstar_c": (R, nf),
                  "lstar_sub": (R, nf), "lstar_sup": (R, nf),
                  "Iplus": (R, nf, na), "Iminus": (R, nf, na), "H": (R, nf), "Iemerg": (nb, nf, na)}
        out = dict(out or {})
        ptrs = {}
        for bit, name in OUTPUT_NAMES.items():
            if self.outputs & bit:
                if name not in out:
                    out[name] = torch.empty(shapes[name], dtype=self.dtype, device=tau.device)
                self._want(out[name], shapes[name], self.dtype, name)
                ptrs[name] = _ptr(out[name])
        fo = FsOut(**ptrs)
        self.ctx._check(self.lib.pprt_formal_solution(self.h, C.byref(fin), C.byref(fo)),
                        "formal_solution")
        return out

    # ------------------------------------------------ emergent intensity + adjoint
    def adjoint_workspace_bytes(self, checkpoint_interval: int = 16) -> int:
        n = C.c_size_t()
        self.ctx._check(self.lib.pprt_plan_adjoint_workspace_bytes(self.h, int(checkpoint_interval),
                                                                   C.byref(n)), "adjoint_workspace_bytes")
        return n.value

    def emergent_intensity(self, tau, q, Sg, Bbot=None, Bbot_prev=None, Ibot=None,
                           checkpoint_interval: int = 16, workspace=None):
        """pprt_emergent_intensity: returns (Iemerg [nb, nf, na], checkpoint workspace)."""
        import torch
        fin = self.fs_in(tau, q, Sg, Bbot, Bbot_prev, None, Ibot)
        nbytes = self.adjoint_workspace_bytes(checkpoint_interval)
        if workspace is None:
            workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=tau.device)
        elif workspace.numel() * workspace.element_size() < nbytes:
            raise ValueError(f"checkpoint workspace needs {nbytes} bytes")
        Iem = torch.empty((self.nb, self.nf, self.na), dtype=self.dtype, device=tau.device)
        self.ctx._check(self.lib.pprt_emergent_intensity(self.h, C.byref(fin), int(checkpoint_interval),
                                                         _ptr(Iem), _ptr(workspace)),
                        "emergent_intensity")
        return Iem, workspace

    def formal_solution_vjp(self, tau, q, Sg, gIemerg, workspace, Bbot=None, Bbot_prev=None,
                            Ibot=None, checkpoint_interval: int = 16) -> dict:
        """pprt_formal_solution_vjp: dL/dq, dL/dSg and the lower-boundary adjoints."""
        import torch
        fin = self.fs_in(tau, q, Sg, Bbot, Bbot_prev, None, Ibot)
        self._want(gIemerg, (self.nb, self.nf, self.na), self.dtype, "gIemerg")
        R, nf, na, nb, dt, dev = self.rows, self.nf, self.na, self.nb, self.dtype, tau.device
        g = {"dq": torch.empty((R, nf), dtype=dt, device=dev),
             "dSg": torch.empty((R, nf), dtype=dt, device=dev)}
        if self.lower_bc == BC_DIFFUSION:
            g["dBbot"] = torch.empty((nb, nf), dtype=dt, device=dev)
            g["dBbot_prev"] = torch.empty((nb, nf), dtype=dt, device=dev)
        else:
            g["dIbot"] = torch.empty((nb, nf, na), dtype=dt, device=dev)
        fg = FsGrad(**{k: _ptr(v) for k, v in g.items()})
        self.ctx._check(self.lib.pprt_formal_solution_vjp(self.h, C.byref(fin), int(checkpoint_interval),
                                                          _ptr(gIemerg), C.byref(fg), _ptr(workspace)),
                        "formal_solution_vjp")
        return g

    def formal_solution_scattering_vjp(self, tau, q, Sg, omega, gIemerg, Bbot=None, Bbot_prev=None,
                                       Itop=None, Ibot=None, workspace=None) -> dict:
        """pprt_formal_solution_scattering_vjp: dL/dq, dL/dSg and the lower-boundary
        adjoints of the emergent intensity with in-layer scattering (omega and
        Itop held fixed).  The returned dict keeps the workspace under
        "_workspace" for reuse."""
        import torch
        fin = self.fs_in(tau, q, Sg, Bbot, Bbot_prev, Itop, Ibot)
        self._want(omega, (self.rows, self.nf), self.dtype, "omega")
        self._want(gIemerg, (self.nb, self.nf, self.na), self.dtype, "gIemerg")
        R, nf, na, nb, dt, dev = self.rows, self.nf, self.na, self.nb, self.dtype, tau.device
        if workspace is None:
            nbytes = C.c_size_t()
            self.ctx._check(self.lib.pprt_plan_scattering_vjp_workspace_bytes(self.h, C.byref(nbytes)),
                            "scattering_vjp_workspace_bytes")
            workspace = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=dev)
        g = {"dq": torch.empty((R, nf), dtype=dt, device=dev),
             "dSg": torch.empty((R, nf), dtype=dt, device=dev)}
        if self.lower_bc == BC_DIFFUSION:
            g["dBbot"] = torch.empty((nb, nf), dtype=dt, device=dev)
            g["dBbot_prev"] = torch.empty((nb, nf), dtype=dt, device=dev)
        else:
            g["dIbot"] = torch.empty((nb, nf, na), dtype=dt, device=dev)
        fg = FsGrad(**{k: _ptr(v) for k, v in g.items()})
        self.ctx._check(self.lib.pprt_formal_solution_scattering_vjp(self.h, C.byref(fin), _ptr(omega),
                                                                     _ptr(gIemerg), C.byref(fg),
                                                                     _ptr(workspace)),
                        "formal_solution_scattering_vjp")
        g["_workspace"] = workspace
        return g

    def set_thick_mode(self, mode: int):
        """pprt_plan_set_thick_mode: THICK_RULE (default), THICK_NEVER or
        THICK_ALWAYS for the FP64 eliminations of the FP32-bulk scattering path."""
        self.ctx._check(self.lib.pprt_plan_set_thick_mode(self.h, int(mode)), "set_thick_mode")

    def formal_solution_scattering(self, tau, q, Sg, omega, Bbot=None, Bbot_prev=None, Itop=None,
                                   Ibot=None, out: dict | None = None, workspace=None) -> dict:
        """pprt_formal_solution_scattering (in-layer coherent isotropic scattering)."""
        import torch
        fin = self.fs_in(tau, q, Sg, Bbot, Bbot_prev, Itop, Ibot)
        self._want(omega, (self.rows, self.nf), self.dtype, "omega")
        R, nf, na, nb = self.rows, self.nf, self.na, self.nb
        shapes = {"J": (R, nf), "JmS": (R, nf), "lstar": (R, nf), "lstar_c": (R, nf),
                  "lstar_sub": (R, nf), "lstar_sup": (R, nf),
                  "Iplus": (R, nf, na), "Iminus": (R, nf, na), "H": (R, nf), "Iemerg": (nb, nf, na)}
        out = dict(out or {})
        ptrs = {}
        for bit, name in OUTPUT_NAMES.items():
            if self.outputs & bit:
                if name not in out:
                    out[name] = torch.empty(shapes[name], dtype=self.dtype, device=tau.device)
                self._want(out[name], shapes[name], self.dtype, name)
                ptrs[name] = _ptr(out[name])
        nbytes = C.c_size_t()
        self.ctx._check(self.lib.pprt_plan_scattering_workspace_bytes(self.h, C.byref(nbytes)),
                        "scattering_workspace_bytes")
        if workspace is None:
            workspace = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=tau.device)
        fo = FsOut(**ptrs)
        self.ctx._check(self.lib.pprt_formal_solution_scattering(
            self.h, C.byref(fin), _ptr(omega), C.byref(fo), _ptr(workspace)), "formal_solution_scattering")
        out["_workspace"] = workspace
        return out

    def two_level(self, eps, B, wphi):
        import torch
        self._want(eps, (self.nb,), torch.float64, "eps")
        self._want(B, (self.rows,), torch.float64, "B")
        self._want(wphi, (self.nf,), self.dtype, "wphi")
        return TwoLevel(_ptr(eps), _ptr(B), _ptr(wphi))

    def two_level_ali_step(self, tau, q, S, eps, B, wphi, max_rel, active=None, Itop=None,
                           Ibot=None):
        """pprt_two_level_ali_step: one formal solution + OS update, S in place."""
        import torch
        fin = self.fs_in(tau, q, None, None, None, Itop, Ibot)
        at = self.two_level(eps, B, wphi)
        self._want(S, (self.rows,), torch.float64, "S")
        self._want(max_rel, (self.nb,), torch.float64, "max_rel")
        if active is not None:
            self._want(active, (self.nb,), torch.int32, "active")
        self.ctx._check(self.lib.pprt_two_level_ali_step(
            self.h, C.byref(fin), C.byref(at), _ptr(S), _ptr(max_rel), _ptr(active),
            _ptr(self.workspace())), "two_level_ali_step")

    def two_level_graph(self, tau, q, S, eps, B, wphi, max_rel, steps=1, active=None, Itop=None,
                        Ibot=None):
        """pprt_two_level_graph_create: `steps` ALI steps captured once; the
        returned StepGraph replays them with .launch().  Keeps the tensors
        alive for the graph's lifetime."""
        import torch
        fin = self.fs_in(tau, q, None, None, None, Itop, Ibot)
        at = self.two_level(eps, B, wphi)
        self._want(S, (self.rows,), torch.float64, "S")
        self._want(max_rel, (self.nb,), torch.float64, "max_rel")
        if active is not None:
            self._want(active, (self.nb,), torch.int32, "active")
        ws = self.workspace()
        h = C.c_void_p()
        self.ctx._check(self.lib.pprt_two_level_graph_create(
            self.h, C.byref(fin), C.byref(at), _ptr(S), _ptr(max_rel), _ptr(active), _ptr(ws),
            int(steps), C.byref(h)), "two_level_graph_create")
        return StepGraph(self, h, (tau, q, S, eps, B, wphi, max_rel, active, Itop, Ibot, ws))

    def two_level_ali_step_noalloc(self, tau, q, S, eps, B, wphi, max_rel, active=None, Itop=None,
                                   Ibot=None):
        """pprt_two_level_ali_step_noalloc: the same step with the library's
        static scratch instead of a workspace (nothing is allocated)."""
        import torch
        fin = self.fs_in(tau, q, None, None, None, Itop, Ibot)
        at = self.two_level(eps, B, wphi)
        self._want(S, (self.rows,), torch.float64, "S")
        self._want(max_rel, (self.nb,), torch.float64, "max_rel")
        if active is not None:
            self._want(active, (self.nb,), torch.int32, "active")
        self.ctx._check(self.lib.pprt_two_level_ali_step_noalloc(
            self.h, C.byref(fin), C.byref(at), _ptr(S), _ptr(max_rel), _ptr(active)),
            "two_level_ali_step_noalloc")

    def two_level_ali_step_continuum(self, tau, q, S, eps, B, wphi, pfrac, sg_const, omega,
                                     Bbot, Bbot_prev, max_rel, active=None, Itop=None, Ibot=None,
                                     workspace=None):
        """pprt_two_level_ali_step_continuum: S^g assembly, formal solution
        (with in-layer scattering if omega is given), profile quadratures and
        the OS update, S in place."""
        import torch
        fin = self.fs_in(tau, q, None, Bbot, Bbot_prev, Itop, Ibot)
        at = self.two_level(eps, B, wphi)
        for name, t in (("pfrac", pfrac), ("sg_const", sg_const)):
            self._want(t, (self.rows, self.nf), self.dtype, name)
        if omega is not None:
            self._want(omega, (self.rows, self.nf), self.dtype, "omega")
        self._want(S, (self.rows,), torch.float64, "S")
        self._want(max_rel, (self.nb,), torch.float64, "max_rel")
        if workspace is None:
            nbytes = C.c_size_t()
            self.ctx._check(self.lib.pprt_plan_continuum_workspace_bytes(self.h, C.byref(nbytes)),
                            "continuum_workspace_bytes")
            if getattr(self, "_cws", None) is None or self._cws.numel() < nbytes.value:
                self._cws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=S.device)
            workspace = self._cws
        ct = Continuum(_ptr(pfrac), _ptr(sg_const), _ptr(omega))
        self.ctx._check(self.lib.pprt_two_level_ali_step_continuum(
            self.h, C.byref(fin), C.byref(at), C.byref(ct), _ptr(S), _ptr(max_rel), _ptr(active),
            _ptr(workspace)), "two_level_ali_step_continuum")

    # ------------------------------------------------------ multilevel
    def _want_atom(self, atom):
        if not isinstance(getattr(atom, "struct", None), Atom):
            raise TypeError("atom must be a DeviceAtom")
        if atom.rows != self.rows or atom.nf != self.nf:
            raise ValueError(f"atom was built for {atom.rows} rows and {atom.nf} frequencies, "
                             f"the plan has {self.rows} and {self.nf}")
        return atom

    def nlte_opacity(self, atom, pops):
        import torch
        R, nf = self.rows, self.nf
        self._want_atom(atom)
        self._want(pops, (R, atom.nlev), torch.float64, "pops")
        q = torch.empty((R, nf), dtype=torch.float64, device=pops.device)
        om = torch.empty_like(q)
        Sg = torch.empty_like(q)
        self.ctx._check(self.lib.pprt_nlte_opacity(self.h, C.byref(atom.struct), _ptr(pops), _ptr(q),
                                                   _ptr(om), _ptr(Sg)), "nlte_opacity")
        return q, om, Sg

    def rates_assemble(self, atom, pops_old, J, lstar):
        import torch
        self._want_atom(atom)
        self._want(pops_old, (self.rows, atom.nlev), torch.float64, "pops_old")
        self._want(J, (self.rows, self.nf), torch.float64, "J")
        self._want(lstar, (self.rows, self.nf), torch.float64, "lstar")
        shp = (self.rows, atom.ntr)
        out = [torch.empty(shp, dtype=torch.float64, device=pops_old.device) for _ in range(3)]
        self.ctx._check(self.lib.pprt_rates_assemble(
            self.h, C.byref(atom.struct), _ptr(pops_old), _ptr(J), _ptr(lstar), *[_ptr(t) for t in out]),
            "rates_assemble")
        return tuple(out)

    def rates_solve(self, atom, pops_old, dRlu, dRul, Rsul):
        import torch
        self._want_atom(atom)
        self._want(pops_old, (self.rows, atom.nlev), torch.float64, "pops_old")
        for name, t in (("dRlu", dRlu), ("dRul", dRul), ("Rsul", Rsul)):
            self._want(t, (self.rows, atom.ntr), torch.float64, name)
        pn = torch.empty_like(pops_old)
        mx = torch.empty(self.nb, dtype=torch.float64, device=pops_old.device)
        self.ctx._check(self.lib.pprt_rates_solve(
            self.h, C.byref(atom.struct), _ptr(pops_old), _ptr(dRlu), _ptr(dRul), _ptr(Rsul), _ptr(pn),
            _ptr(mx)), "rates_solve")
        return pn, mx

    def _nlte_args(self, tau, atom, pops, Itop):
        import torch
        self._want_atom(atom)
        self._want(tau, (self.rows,), torch.float64, "tau")
        self._want(pops, (self.rows, atom.nlev), torch.float64, "pops")
        if Itop is not None:
            self._want(Itop, (self.nb, self.nf, self.na), torch.float64, "Itop")
        fin = FsIn(_ptr(tau), None, None, _ptr(Itop), None, None, None)
        nbytes = C.c_size_t()
        self.ctx._check(self.lib.pprt_plan_nlte_workspace_bytes(self.h, atom.nlev, atom.ntr,
                                                                C.byref(nbytes)), "nlte_workspace_bytes")
        if getattr(self, "_nws", None) is None or self._nws.numel() < nbytes.value:
            self._nws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=tau.device)
        return fin

    def nlte_step(self, tau, atom, pops, max_rel, Itop=None):
        import torch
        fin = self._nlte_args(tau, atom, pops, Itop)
        self._want(max_rel, (self.nb,), torch.float64, "max_rel")
        self.ctx._check(self.lib.pprt_nlte_step(self.h, C.byref(fin), C.byref(atom.struct), _ptr(pops),
                                                _ptr(max_rel), _ptr(self._nws)), "nlte_step")

    def nlte_solve(self, tau, atom, pops, tol=1e-8, max_iter=200, iters_per_sync=8, iters=None,
                   Itop=None, raise_not_converged=True):
        """pprt_nlte_solve: the multilevel loop to tolerance; pops in place.
        Returns the report dict."""
        import torch
        fin = self._nlte_args(tau, atom, pops, Itop)
        if iters is not None:
            self._want(iters, (self.nb,), torch.int32, "iters")
        ctl = AliCtl(float(tol), int(max_iter), int(iters_per_sync), 0, 0)
        rep = AliReport()
        st = self.lib.pprt_nlte_solve(self.h, C.byref(fin), C.byref(atom.struct), C.byref(ctl),
                                      _ptr(pops), _ptr(iters), C.byref(rep), _ptr(self._nws))
        report = {"iterations": rep.iterations, "n_converged": rep.n_converged,
                  "max_rel": rep.max_rel, "status": STATUS.get(st, st)}
        if st == 6 and not raise_not_converged:
            return report
        self.ctx._check(st, "nlte_solve")
        return report

    # ------------------------------------------------ ALI checkpoint / resume
    def ali_state_export(self, S) -> np.ndarray:
        """pprt_ali_state_export: a host byte image of S and the iteration
        state held in this plan's workspace."""
        import torch
        self._want(S, (self.rows,), torch.float64, "S")
        n = C.c_size_t()
        self.ctx._check(self.lib.pprt_ali_state_bytes(self.h, C.byref(n)), "ali_state_bytes")
        buf = np.zeros(n.value, dtype=np.uint8)
        self.ctx._check(self.lib.pprt_ali_state_export(self.h, _ptr(S), _ptr(self.workspace()),
                                                       C.c_void_p(buf.ctypes.data), n.value),
                        "ali_state_export")
        return buf

    def ali_state_import(self, image, S):
        """pprt_ali_state_import: restore S and this plan's workspace state."""
        import torch
        self._want(S, (self.rows,), torch.float64, "S")
        image = np.ascontiguousarray(image, dtype=np.uint8)
        self.ctx._check(self.lib.pprt_ali_state_import(self.h, C.c_void_p(image.ctypes.data),
                                                       int(image.size), _ptr(S), _ptr(self.workspace())),
                        "ali_state_import")

    def two_level_moments(self, tau, q, S, eps, B, wphi, active=None, Itop=None, Ibot=None):
        """pprt_two_level_moments: the formal-solution half of an ALI step."""
        import torch
        fin = self.fs_in(tau, q, None, None, None, Itop, Ibot)
        at = self.two_level(eps, B, wphi)
        self._want(S, (self.rows,), torch.float64, "S")
        self.ctx._check(self.lib.pprt_two_level_moments(
            self.h, C.byref(fin), C.byref(at), _ptr(S), _ptr(active), _ptr(self.workspace())),
            "two_level_moments")

    def two_level_update(self, S, eps, B, wphi, max_rel, active=None):
        """pprt_two_level_update: the float64 update half of an ALI step."""
        import torch
        at = self.two_level(eps, B, wphi)
        self._want(S, (self.rows,), torch.float64, "S")
        self._want(max_rel, (self.nb,), torch.float64, "max_rel")
        self.ctx._check(self.lib.pprt_two_level_update(
            self.h, C.byref(at), _ptr(S), _ptr(max_rel), _ptr(active), _ptr(self.workspace())),
            "two_level_update")

    def two_level_ali(self, tau, q, S, eps, B, wphi, tol=1e-8, max_iter=20000,
                      iters_per_sync=64, use_graph=False, iters=None, Itop=None, Ibot=None,
                      raise_not_converged=True, resume=False):
        """pprt_two_level_ali: iterate to convergence; returns the report dict."""
        import torch
        fin = self.fs_in(tau, q, None, None, None, Itop, Ibot)
        at = self.two_level(eps, B, wphi)
        self._want(S, (self.rows,), torch.float64, "S")
        if iters is not None:
            self._want(iters, (self.nb,), torch.int32, "iters")
        ctl = AliCtl(float(tol), int(max_iter), int(iters_per_sync), int(bool(use_graph)),
                     int(bool(resume)))
        rep = AliReport()
        st = self.lib.pprt_two_level_ali(self.h, C.byref(fin), C.byref(at), C.byref(ctl), _ptr(S),
                                         _ptr(iters), C.byref(rep), _ptr(self.workspace()))
        report = {"iterations": rep.iterations, "n_converged": rep.n_converged,
                  "max_rel": rep.max_rel, "status": STATUS.get(st, st)}
        if st == 6 and not raise_not_converged:
            return report
        self.ctx._check(st, "two_level_ali")
        return report


    # ------------------------------------------------ approximate operator
    def set_operator(self, lstar: int = LSTAR_DIAG, ng: bool = False):
        """pprt_plan_set_operator; resizes (and drops) the cached workspace."""
        self.ctx._check(self.lib.pprt_plan_set_operator(self.h, int(lstar), int(bool(ng))),
                        "set_operator")
        nb = C.c_size_t()
        self.ctx._check(self.lib.pprt_plan_workspace_bytes(self.h, C.byref(nb)), "workspace_bytes")
        self.workspace_bytes = nb.value
        self._ws = None

    def two_level_reset(self):
        self.ctx._check(self.lib.pprt_two_level_reset(self.h, _ptr(self.workspace())), "two_level_reset")

    # ------------------------------------------------ launch shape / autotuner
    def set_launch(self, waves_per_block: int, persistent_waves_per_cu: int = 0):
        self.ctx._check(self.lib.pprt_plan_set_launch(self.h, int(waves_per_block),
                                                      int(persistent_waves_per_cu)), "set_launch")

    def get_launch(self):
        a, b = C.c_int32(), C.c_int32()
        self.ctx._check(self.lib.pprt_plan_get_launch(self.h, C.byref(a), C.byref(b)), "get_launch")
        return a.value, b.value

    def autotune(self, tau, q, S, eps, B, wphi, force=False, Itop=None, Ibot=None) -> dict:
        """pprt_plan_autotune on these inputs; returns the report."""
        import torch
        fin = self.fs_in(tau, q, None, None, None, Itop, Ibot)
        at = self.two_level(eps, B, wphi)
        self._want(S, (self.rows,), torch.float64, "S")
        rep = TuneReport()
        self.ctx._check(self.lib.pprt_plan_autotune(self.h, C.byref(fin), C.byref(at), _ptr(S),
                                                    _ptr(self.workspace()), int(bool(force)),
                                                    C.byref(rep)), "autotune")
        return {k: getattr(rep, k) for k, _ in TuneReport._fields_}


class StepGraph:
    """A captured sequence of ALI steps (pprt_two_level_graph_create)."""

    def __init__(self, plan, h, keep):
        self.plan, self.h, self._keep = plan, h, keep

    def launch(self):
        self.plan.ctx._check(self.plan.lib.pprt_graph_launch(self.h), "graph_launch")

    def close(self):
        if getattr(self, "h", None):
            self.plan.lib.pprt_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SphPlan:
    """Ragged batch of spherical atmospheres (see pprt_sph_plan_create): radii
    r [rows] (host, decreasing inward per atmosphere), n_core core rays plus
    one tangent ray per shell."""

    OUTPUTS = {OUT_J: "J", OUT_JMS: "JmS", OUT_LSTAR: "lstar", OUT_LSTAR_C: "lstar_c", OUT_H: "H"}

    def __init__(self, ctx: Context, nd, nf: int, r, n_core: int, precision: int = FP32,
                 lower_bc: int = BC_DIFFUSION, outputs: int = OUT_JMS | OUT_LSTAR_C):
        import torch
        self.ctx, self.lib = ctx, ctx.lib
        self.nd = np.ascontiguousarray(np.asarray(nd, dtype=np.int32))
        self.nf, self.precision, self.n_core = int(nf), int(precision), int(n_core)
        self.lower_bc, self.outputs = int(lower_bc), int(outputs)
        self._r = np.ascontiguousarray(np.asarray(r, dtype=np.float64))
        if self._r.shape != (int(self.nd.sum()),):
            raise ValueError(f"r must have shape ({int(self.nd.sum())},)")
        h = C.c_void_p()
        ctx._check(self.lib.pprt_sph_plan_create(
            ctx.h, int(self.nd.shape[0]), self.nd.ctypes.data_as(C.POINTER(C.c_int32)), self.nf,
            self.precision, self.lower_bc, self.outputs, self._r.ctypes.data_as(C.POINTER(C.c_double)),
            self.n_core, C.byref(h)), "sph_plan_create")
        self.h = h
        rows, nr, pairs = C.c_int64(), C.c_int32(), C.c_int64()
        ctx._check(self.lib.pprt_sph_plan_info(h, C.byref(rows), C.byref(nr), C.byref(pairs)),
                   "sph_plan_info")
        self.rows, self.nrays, self.pairs = rows.value, nr.value, pairs.value
        nb = C.c_size_t()
        ctx._check(self.lib.pprt_sph_plan_workspace_bytes(h, C.byref(nb)), "sph_workspace_bytes")
        self.workspace_bytes = nb.value
        self.dtype = torch.float64 if self.precision == FP64 else torch.float32
        self._ws = None

    @property
    def nb(self) -> int:
        return int(self.nd.shape[0])

    def workspace(self):
        import torch
        if self._ws is None:
            self._ws = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8,
                                   device=f"cuda:{self.ctx.device}")
        return self._ws

    def close(self):
        if getattr(self, "h", None):
            self.lib.pprt_sph_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    _want = Plan._want

    def fs_in(self, tau, q, Sg=None, Bbot=None, Bbot_prev=None, Itop=None, Ibot=None):
        import torch
        R, nf, nb, dt = self.rows, self.nf, self.nb, self.dtype
        self._want(tau, (R,), torch.float64, "tau")
        self._want(q, (R, nf), dt, "q")
        if Sg is not None:
            self._want(Sg, (R, nf), dt, "Sg")
        for name, t in (("Bbot", Bbot), ("Bbot_prev", Bbot_prev), ("Itop", Itop), ("Ibot", Ibot)):
            if t is not None:
                self._want(t, (nb, nf), dt, name)
        return FsIn(_ptr(tau), _ptr(q), _ptr(Sg), _ptr(Itop), _ptr(Bbot), _ptr(Bbot_prev), _ptr(Ibot))

    def formal_solution(self, tau, q, Sg, Bbot=None, Bbot_prev=None, Itop=None, Ibot=None) -> dict:
        """pprt_sph_formal_solution: returns a dict of the requested [rows, nf] outputs."""
        import torch
        fin = self.fs_in(tau, q, Sg, Bbot, Bbot_prev, Itop, Ibot)
        out, ptrs = {}, {}
        for bit, name in self.OUTPUTS.items():
            if self.outputs & bit:
                out[name] = torch.empty((self.rows, self.nf), dtype=self.dtype, device=tau.device)
                ptrs[name] = _ptr(out[name])
        fo = FsOut(**ptrs)
        self.ctx._check(self.lib.pprt_sph_formal_solution(self.h, C.byref(fin), C.byref(fo)),
                        "sph_formal_solution")
        return out

    def _two_level(self, eps, B, wphi, S, active):
        import torch
        self._want(eps, (self.nb,), torch.float64, "eps")
        self._want(B, (self.rows,), torch.float64, "B")
        self._want(wphi, (self.nf,), self.dtype, "wphi")
        self._want(S, (self.rows,), torch.float64, "S")
        if active is not None:
            self._want(active, (self.nb,), torch.int32, "active")
        return TwoLevel(_ptr(eps), _ptr(B), _ptr(wphi))

    def two_level_ali_step(self, tau, q, S, eps, B, wphi, max_rel, active=None, Itop=None, Ibot=None):
        """pprt_sph_two_level_ali_step: one spherical formal solution + OS update, S in place."""
        import torch
        fin = self.fs_in(tau, q, None, None, None, Itop, Ibot)
        at = self._two_level(eps, B, wphi, S, active)
        self._want(max_rel, (self.nb,), torch.float64, "max_rel")
        self.ctx._check(self.lib.pprt_sph_two_level_ali_step(
            self.h, C.byref(fin), C.byref(at), _ptr(S), _ptr(max_rel), _ptr(active),
            _ptr(self.workspace())), "sph_two_level_ali_step")

    def two_level_moments(self, tau, q, S, eps, B, wphi, active=None, Itop=None, Ibot=None):
        """pprt_sph_two_level_moments: the sweep half of the step."""
        fin = self.fs_in(tau, q, None, None, None, Itop, Ibot)
        at = self._two_level(eps, B, wphi, S, active)
        self.ctx._check(self.lib.pprt_sph_two_level_moments(
            self.h, C.byref(fin), C.byref(at), _ptr(S), _ptr(active), _ptr(self.workspace())),
            "sph_two_level_moments")

    def two_level_update(self, S, eps, B, wphi, max_rel, active=None):
        """pprt_sph_two_level_update: the float64 update half of the step."""
        import torch
        at = self._two_level(eps, B, wphi, S, active)
        self._want(max_rel, (self.nb,), torch.float64, "max_rel")
        self.ctx._check(self.lib.pprt_sph_two_level_update(
            self.h, C.byref(at), _ptr(S), _ptr(max_rel), _ptr(active), _ptr(self.workspace())),
            "sph_two_level_update")


class DeviceAtom:
    """A workloads.MultiLevelAtom resident on the device (tables as int32,
    everything else float64) plus the pprt_atom struct pointing at it."""

    def __init__(self, atom, device="cuda:0"):
        import torch
        i32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32), device=device)
        f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)
        self.nlev, self.ntr = int(atom.nl), int(atom.nt)
        self.t = dict(lower=i32(atom.lo), upper=i32(atom.up), k0=i32(atom.k0), k1=i32(atom.k1),
                      owner=i32(atom.owner), sigma=f64(atom.sigma), bfac=f64(atom.bfac), W=f64(atom.W),
                      G=f64(atom.Gst), Bnu=f64(atom.Bnu), kc=f64(atom.kc), sc=f64(atom.sc),
                      ntot=f64(atom.ntot), Cul=f64(atom.Cul), Clu=f64(atom.Clu))
        voigt = getattr(atom, "line_a", None) is not None
        if voigt:
            self.t.update(nu=f64(atom.nu), line_nu0=f64(atom.line_nu0), line_s=f64(atom.line_s),
                          line_a=f64(atom.line_a), dopp=f64(atom.dopp))
        self.tau = f64(atom.tau)
        self.nstar = f64(atom.nstar)
        self.rows, self.nf = int(self.t["G"].shape[0]), int(self.t["owner"].shape[0])
        names = ["lower", "upper", "k0", "k1", "owner", "sigma", "bfac", "W", "G", "Bnu", "kc", "sc",
                 "ntot", "Cul", "Clu"]
        extra = ["nu", "line_nu0", "line_s", "line_a", "dopp"]
        self.struct = Atom(self.nlev, self.ntr, *[_ptr(self.t[n]) for n in names],
                           *[_ptr(self.t[n]) if voigt else None for n in extra])


@dataclass
class DeviceBatch:
    """A TwoLevelBatch's arrays resident on the device in the plan's precision."""
    tau: object
    q: object
    S: object
    B: object
    eps: object
    wphi: object
    Bbot: object
    Bbot_prev: object


def upload_two_level(batch, precision: int, device="cuda:0") -> DeviceBatch:
    """Copy a workloads.TwoLevelBatch to the device (no arithmetic beyond
    gathering the boundary values of B per atmosphere)."""
    import torch
    dt = torch.float64 if precision == FP64 else torch.float32
    off = batch.off
    last = off[1:] - 1
    Bb = np.repeat(batch.B[last][:, None], batch.nf, axis=1)
    Bp = np.repeat(batch.B[last - 1][:, None], batch.nf, axis=1)
    t = lambda a, d: torch.as_tensor(np.ascontiguousarray(a), dtype=d, device=device)
    return DeviceBatch(
        tau=t(batch.tau, torch.float64), q=t(batch.q, dt), S=t(batch.S_trial, torch.float64),
        B=t(batch.B, torch.float64), eps=t(batch.eps, torch.float64),
        wphi=t(batch.wnu * batch.phi, dt), Bbot=t(Bb, dt), Bbot_prev=t(Bp, dt))


def _vox_grid(r, nt, np_):
    r = np.ascontiguousarray(np.asarray(r, dtype=np.float64))
    return VoxGrid(int(r.shape[0] - 1), int(nt), int(np_), r.ctypes.data_as(C.POINTER(C.c_double))), r


def vox_geometry_host(r, nt, np_, n_mu, n_phi, spacing=0.0):
    """pprt_vox_geometry_host: the characteristics the voxel plan builds, on
    the host only.  Returns a dict of numpy arrays (ray_seg0, ray_dir,
    ray_core, seg_ijk, seg_ell, seg_wn)."""
    lib = load_library()
    g, keep = _vox_grid(r, nt, np_)
    nr_, ns_ = C.c_int64(), C.c_int64()
    st = lib.pprt_vox_geometry_host(C.byref(g), int(n_mu), int(n_phi), float(spacing), C.byref(nr_), C.byref(ns_),
                                    None, None, None, None, None, None)
    if st != 0:
        raise PprtError(st, "vox_geometry_host")
    out = {"ray_seg0": np.zeros(nr_.value + 1, np.int64), "ray_dir": np.zeros(nr_.value, np.int32),
           "ray_core": np.zeros(nr_.value, np.uint8), "seg_ijk": np.zeros(ns_.value, np.uint32),
           "seg_ell": np.zeros(ns_.value), "seg_wn": np.zeros(ns_.value)}
    st = lib.pprt_vox_geometry_host(C.byref(g), int(n_mu), int(n_phi), float(spacing), C.byref(nr_), C.byref(ns_),
                                    *(out[k].ctypes.data for k in ("ray_seg0", "ray_dir", "ray_core", "seg_ijk",
                                                                   "seg_ell", "seg_wn")))
    if st != 0:
        raise PprtError(st, "vox_geometry_host")
    del keep
    return out


class VoxPlan:
    """3D full characteristics on a spherical voxel grid (pprt_vox_plan_create):
    radial edges r [nr + 1] (host), nt x np angular voxels, n_mu x n_phi
    directions, lattice spacing (<= 0: default), nf frequencies."""

    def __init__(self, ctx: Context, r, nt: int, np_: int, n_mu: int, n_phi: int, nf: int,
                 precision: int = FP32, spacing: float = 0.0):
        import torch
        self.ctx, self.lib = ctx, ctx.lib
        g, self._r = _vox_grid(r, nt, np_)
        self.nr, self.nt, self.np_ = g.nr, g.nt, g.np
        self.nf, self.precision = int(nf), int(precision)
        h = C.c_void_p()
        ctx._check(self.lib.pprt_vox_plan_create(ctx.h, C.byref(g), int(n_mu), int(n_phi), float(spacing), self.nf,
                                                 self.precision, C.byref(h)), "vox_plan_create")
        self.h = h
        info = VoxInfo()
        ctx._check(self.lib.pprt_vox_plan_info(h, C.byref(info)), "vox_plan_info")
        self.info = {k: getattr(info, k) for k, _ in VoxInfo._fields_}
        self.nvox, self.ndir = int(info.nvox), int(info.ndir)
        d = np.zeros((self.ndir, 3))
        w = np.zeros(self.ndir)
        ctx._check(self.lib.pprt_vox_directions(h, d.ctypes.data_as(C.POINTER(C.c_double)),
                                                w.ctypes.data_as(C.POINTER(C.c_double))), "vox_directions")
        self.dirs, self.w = d, w
        nb = C.c_size_t()
        ctx._check(self.lib.pprt_vox_ali_workspace_bytes(h, C.byref(nb)), "vox_ali_workspace_bytes")
        self.ali_workspace_bytes = nb.value
        self.dtype = torch.float64 if self.precision == FP64 else torch.float32
        self._ws = None

    _want = Plan._want

    def formal_solution(self, chi, S, I_out=None, I_core=None, flux=False, lstar=False, out=None):
        """J [nvox, nf] (float64) and, if asked, the flux [nvox, 3, nf]
        (Cartesian) and Lambda* [nvox, 27, nf]."""
        import torch
        V, nf, dt = self.nvox, self.nf, self.dtype
        self._want(chi, (V, nf), dt, "chi")
        self._want(S, (V, nf), dt, "S")
        if I_out is not None:
            self._want(I_out, (nf,), dt, "I_out")
        if I_core is not None:
            self._want(I_core, (nf,), dt, "I_core")
        dev = chi.device
        out = dict(out or {})
        out.setdefault("J", torch.empty((V, nf), dtype=torch.float64, device=dev))
        self._want(out["J"], (V, nf), torch.float64, "J")
        if flux:
            out.setdefault("flux", torch.empty((V, 3, nf), dtype=torch.float64, device=dev))
            self._want(out["flux"], (V, 3, nf), torch.float64, "flux")
        if lstar:
            out.setdefault("lstar", torch.empty((V, 27, nf), dtype=torch.float64, device=dev))
            self._want(out["lstar"], (V, 27, nf), torch.float64, "lstar")
        self.ctx._check(self.lib.pprt_vox_formal_solution(
            self.h, _ptr(chi), _ptr(S), _ptr(I_out), _ptr(I_core), _ptr(out["J"]),
            _ptr(out.get("flux") if flux else None), _ptr(out.get("lstar") if lstar else None)),
            "vox_formal_solution")
        return out

    def ali_step(self, chi, S, B, eps, max_rel, I_out=None, I_core=None, workspace=None):
        """pprt_vox_ali_step: S (float64 [nvox, nf]) in place; max_rel float64 [1]."""
        import torch
        V, nf, dt = self.nvox, self.nf, self.dtype
        self._want(chi, (V, nf), dt, "chi")
        self._want(S, (V, nf), torch.float64, "S")
        self._want(B, (V, nf), torch.float64, "B")
        self._want(eps, (V,), torch.float64, "eps")
        self._want(max_rel, (1,), torch.float64, "max_rel")
        if I_out is not None:
            self._want(I_out, (nf,), dt, "I_out")
        if I_core is not None:
            self._want(I_core, (nf,), dt, "I_core")
        if workspace is None:
            if self._ws is None:
                self._ws = torch.empty(max(self.ali_workspace_bytes, 256), dtype=torch.uint8, device=S.device)
            workspace = self._ws
        self.ctx._check(self.lib.pprt_vox_ali_step(self.h, _ptr(chi), _ptr(S), _ptr(B), _ptr(eps), _ptr(I_out),
                                                   _ptr(I_core), _ptr(max_rel), _ptr(workspace)), "vox_ali_step")

    def close(self):
        if getattr(self, "h", None):
            self.lib.pprt_vox_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
