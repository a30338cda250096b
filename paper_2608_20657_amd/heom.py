"""Python binding of libheom (include/heom.h): argument marshalling only.

Every step of the hot path runs in the library's HIP kernels; this module
converts Python values to the C structs, passes device pointers of torch
tensors (torch is used for device memory and streams only), and turns error
codes into exceptions. Importing it loads libheom.so and fails loudly if the
library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libheom.so")

HEOM_OK = 0
HEOM_NOBS = 10
HEOM_FP64 = 0
HEOM_FP32 = 1
HEOM_HERMITIAN = 2      # flag OR-ed into precision: every ADO is Hermitian
HEOM_NOALLOC_WORK_BYTES = 64 << 20   # work memory of heom_propagate_noalloc
HEOM_RECON_MAX_N = 4096              # molecules of heom_reconstruct_dense's dense output
HEOM_RECON_R_DOUBLES = 164           # doubles of its five packed slot matrices
HEOM_RECON_CE_ADJOINT = 32           # mask flag: |c><e_1| response = adjoint of the |e_1><c| one
ERRORS = {-1: "E_INVAL", -2: "E_NOMEM", -3: "E_TOO_LARGE", -4: "E_HIP", -5: "E_NONFINITE",
          -6: "E_UNSUPPORTED", -7: "E_STATE", -8: "E_TIMEOUT"}

# every symbol include/heom.h declares
SYMBOLS = ["heom_build_tables", "heom_set_params", "heom_table_info", "heom_upload", "heom_tier0_pure",
           "heom_tier0_operator", "heom_tier0_expand",
           "heom_init_state", "heom_rhs", "heom_propagate", "heom_propagate_noalloc", "heom_observables",
           "heom_export_layout",
           "heom_export_coefficients", "heom_free_tables", "heom_last_error", "heom_version",
           "heom_set_tuning", "heom_get_tuning", "heom_work_status", "heom_params_bytes",
           "heom_upload_params", "heom_batch_create", "heom_batch_set_slot", "heom_batch_clear_slot",
           "heom_batch_device_bytes", "heom_batch_commit", "heom_batch_propagate", "heom_batch_slot_steps",
           "heom_batch_set_graph", "heom_batch_set_interleave", "heom_batch_set_merge", "heom_batch_set_share", "heom_batch_status",
           "heom_batch_free", "heom_reconstruct_dense", "heom_reconstruct_work_bytes"]


class HeomError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("m", ctypes.c_int32), ("L", ctypes.c_int32),
                ("d", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("c", ctypes.POINTER(ctypes.c_double)), ("c_check", ctypes.POINTER(ctypes.c_double)),
                ("nu", ctypes.POINTER(ctypes.c_double)),
                ("eps", ctypes.c_double), ("omega_c", ctypes.c_double), ("g", ctypes.c_double),
                ("kappa", ctypes.c_double), ("terminator", ctypes.c_double)]


class _Tuning(ctypes.Structure):
    _fields_ = [("tile_vars", ctypes.c_int32), ("persistent", ctypes.c_int32), ("xcd_map", ctypes.c_int32),
                ("max_workgroups", ctypes.c_int32), ("spin_limit", ctypes.c_int32),
                ("cache_policy", ctypes.c_int32), ("transposed", ctypes.c_int32), ("compact", ctypes.c_int32)]


class _Sizes(ctypes.Structure):
    _fields_ = [("n_patterns", ctypes.c_int64), ("n_var", ctypes.c_int64), ("n_conn", ctypes.c_int64),
                ("n_tiles", ctypes.c_int64), ("n_categories", ctypes.c_int64),
                ("table_bytes", ctypes.c_int64), ("work_bytes_fp64", ctypes.c_int64),
                ("work_bytes_fp32", ctypes.c_int64), ("tier0_size", ctypes.c_int64),
                ("max_G", ctypes.c_int32), ("tile_vars", ctypes.c_int32), ("hier_gathers", ctypes.c_int64),
                ("rhs_work_bytes", ctypes.c_int64), ("transposed", ctypes.c_int32), ("compact", ctypes.c_int32),
                ("stage_table_bytes", ctypes.c_int64), ("own_entries", ctypes.c_int64),
                ("read_entries", ctypes.c_int64)]


def _load():
    # PyTorch ships its own HIP runtime and loads it by file name. Loading it
    # first makes libheom bind to that same runtime (same soname); loading
    # libheom first would put two HIP/HSA runtimes into the process.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or python paper_2608_20657_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    sig = {
        "heom_build_tables": [ctypes.POINTER(_Problem), ctypes.POINTER(vp)],
        "heom_set_params": [vp, ctypes.POINTER(_Problem)],
        "heom_table_info": [vp, ctypes.POINTER(_Sizes)],
        "heom_upload": [vp, vp, ctypes.c_size_t, vp],
        "heom_tier0_pure": [vp, dp, dp, dp, dp],
        "heom_tier0_operator": [vp, dp, dp],
        "heom_tier0_expand": [vp, dp, dp],
        "heom_init_state": [vp, dp, vp, vp],
        "heom_rhs": [vp, vp, vp, vp, ctypes.c_size_t, ctypes.c_int, vp],
        "heom_propagate": [vp, vp, vp, ctypes.c_size_t, ctypes.c_double, i64, i64, vp, ctypes.c_int, vp],
        "heom_propagate_noalloc": [vp, vp, ctypes.c_double, i64, i64, vp, ctypes.c_int, vp],
        "heom_observables": [vp, vp, vp, vp],
        "heom_export_layout": [vp, ctypes.POINTER(i64), ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
        "heom_export_coefficients": [vp, dp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
        "heom_set_tuning": [vp, ctypes.POINTER(_Tuning)],
        "heom_get_tuning": [vp, ctypes.POINTER(_Tuning)],
        "heom_work_status": [vp, vp, ctypes.c_size_t, vp],
        "heom_params_bytes": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "heom_upload_params": [vp, ctypes.POINTER(_Problem), vp, ctypes.c_size_t, vp],
        "heom_batch_create": [ctypes.c_int32, ctypes.POINTER(vp)],
        "heom_batch_set_slot": [vp, ctypes.c_int32, vp, vp, vp, vp, ctypes.c_size_t, ctypes.c_double, vp,
                                i64, i64],
        "heom_batch_clear_slot": [vp, ctypes.c_int32],
        "heom_batch_device_bytes": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "heom_batch_commit": [vp, vp, ctypes.c_size_t, vp],
        "heom_batch_propagate": [vp, i64, ctypes.c_int, vp],
        "heom_batch_slot_steps": [vp, ctypes.c_int32, ctypes.POINTER(i64)],
        "heom_batch_set_graph": [vp, ctypes.c_int32],
        "heom_batch_set_merge": [vp, ctypes.c_int32],
        "heom_batch_set_interleave": [vp, ctypes.c_int32],
        "heom_batch_status": [vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, vp],
        "heom_batch_set_share": [vp, ctypes.c_int32],
        "heom_reconstruct_dense": [i64, vp, dp, ctypes.c_uint32, vp, ctypes.c_size_t, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.heom_free_tables.argtypes = [vp]
    lib.heom_free_tables.restype = None
    lib.heom_batch_free.argtypes = [vp]
    lib.heom_batch_free.restype = None
    lib.heom_reconstruct_work_bytes.argtypes = [i64]
    lib.heom_reconstruct_work_bytes.restype = ctypes.c_size_t
    lib.heom_last_error.restype = ctypes.c_char_p
    lib.heom_version.restype = ctypes.c_char_p
    return lib


LIB = _load()


def _check(rc: int):
    if rc != HEOM_OK:
        raise HeomError(rc, LIB.heom_last_error().decode())


def _dbl(values: Sequence[float]):
    arr = (ctypes.c_double * len(values))(*values)
    return arr


def _problem_struct(p):
    c = _dbl([x for z in p.c for x in (complex(z).real, complex(z).imag)])
    cc = _dbl([x for z in p.c_check for x in (complex(z).real, complex(z).imag)])
    nu = _dbl([float(x) for x in p.nu])
    s = _Problem(N=int(p.N), m=int(p.m), L=int(p.L), d=int(p.d), reserved=0,
                 c=ctypes.cast(c, ctypes.POINTER(ctypes.c_double)),
                 c_check=ctypes.cast(cc, ctypes.POINTER(ctypes.c_double)),
                 nu=ctypes.cast(nu, ctypes.POINTER(ctypes.c_double)),
                 eps=float(p.eps), omega_c=float(p.omega_c), g=float(p.g),
                 kappa=float(p.kappa), terminator=float(p.terminator))
    return s, (c, cc, nu)


def _ptr(t) -> int:
    """Device (or host) address of a torch tensor or numpy array."""
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return t.ctypes.data


def _stream(stream) -> Optional[int]:
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


class Tables:
    """Owner of one heom_tables handle."""

    def __init__(self, problem):
        self.problem = problem
        s, keep = _problem_struct(problem)
        h = ctypes.c_void_p()
        _check(LIB.heom_build_tables(ctypes.byref(s), ctypes.byref(h)))
        self._h = h
        self.image = None   # device buffer once uploaded

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and LIB is not None:
            LIB.heom_free_tables(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        z = _Sizes()
        _check(LIB.heom_table_info(self._h, ctypes.byref(z)))
        return {name: getattr(z, name) for name, _ in _Sizes._fields_}

    def set_params(self, problem):
        s, keep = _problem_struct(problem)
        _check(LIB.heom_set_params(self._h, ctypes.byref(s)))
        self.problem = problem

    def upload(self, device_buffer, stream=None):
        """Copy the table image into a caller-owned device buffer (a uint8
        torch tensor of at least info()['table_bytes'] bytes)."""
        nbytes = device_buffer.numel() * device_buffer.element_size()
        _check(LIB.heom_upload(self._h, _ptr(device_buffer), nbytes, _stream(stream)))
        self.image = device_buffer

    def tier0_pure(self, a_c: complex, a_pool: complex, a_dist: Sequence[complex] = ()) -> np.ndarray:
        n0 = self.info()["tier0_size"]
        out = np.zeros(2 * n0)
        ac = _dbl([complex(a_c).real, complex(a_c).imag])
        ap = _dbl([complex(a_pool).real, complex(a_pool).imag])
        ad = _dbl([x for z in a_dist for x in (complex(z).real, complex(z).imag)]) if len(a_dist) else None
        _check(LIB.heom_tier0_pure(self._h, ac, ad, ap, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.view(np.complex128)

    def tier0_operator(self, R: np.ndarray) -> np.ndarray:
        """Tier-0 block of a pool-invariant operator given by its
        (d+3)x(d+3) slot matrix R (cavity, distinguished molecules, two pool
        molecules)."""
        ns = self.problem.d + 3
        R = np.ascontiguousarray(np.asarray(R, dtype=np.complex128))
        if R.shape != (ns, ns):
            raise ValueError(f"R must be {ns}x{ns}")
        n0 = self.info()["tier0_size"]
        out = np.zeros(2 * n0)
        Rv = R.view(np.float64)
        _check(LIB.heom_tier0_operator(self._h, Rv.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.view(np.complex128)

    def tier0_expand(self, tier0: np.ndarray) -> np.ndarray:
        """Slot matrix R of the operator whose tier-0 block is `tier0`."""
        ns = self.problem.d + 3
        t0 = np.ascontiguousarray(np.asarray(tier0, dtype=np.complex128)).view(np.float64)
        R = np.zeros((ns, ns), dtype=np.complex128)
        _check(LIB.heom_tier0_expand(self._h, t0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     R.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return R

    def init_state(self, tier0: np.ndarray, y, stream=None):
        t0 = np.ascontiguousarray(np.asarray(tier0, dtype=np.complex128)).view(np.float64)
        _check(LIB.heom_init_state(self._h, t0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(y),
                                   _stream(stream)))

    def rhs(self, y, dy, stream=None, work=None, precision: int = HEOM_FP64):
        """dy = M_u y (complex128 vectors at HEOM_FP64, complex64 at HEOM_FP32,
        HEOM_HERMITIAN OR-able). `work`: a device buffer of at least
        info()['rhs_work_bytes'] bytes, needed without HEOM_HERMITIAN on tables
        with transposed column targets (allocated here if None)."""
        need = self.info()["rhs_work_bytes"] if not (precision & HEOM_HERMITIAN) else 0
        if work is None and need > 0:
            import torch
            work = torch.empty(need, dtype=torch.uint8, device=y.device)
        wbytes = work.numel() * work.element_size() if work is not None else 0
        _check(LIB.heom_rhs(self._h, _ptr(y), _ptr(dy), _ptr(work) if work is not None else None, wbytes,
                            int(precision), _stream(stream)))

    def propagate(self, y, work, dt: float, nsteps: int, obs_every: int = 0, obs=None,
                  precision: int = HEOM_FP64, stream=None):
        wbytes = work.numel() * work.element_size()
        _check(LIB.heom_propagate(self._h, _ptr(y), _ptr(work), wbytes, float(dt), int(nsteps),
                                  int(obs_every), _ptr(obs) if obs is not None else None,
                                  int(precision), _stream(stream)))

    def propagate_noalloc(self, y, dt: float, nsteps: int, obs_every: int = 0, obs=None,
                          precision: int = HEOM_FP64, stream=None):
        """heom_propagate with the library's static work array instead of a
        caller buffer (allocates nothing; calls on one GPU must not overlap)."""
        _check(LIB.heom_propagate_noalloc(self._h, _ptr(y), float(dt), int(nsteps), int(obs_every),
                                          _ptr(obs) if obs is not None else None, int(precision),
                                          _stream(stream)))

    def observables(self, y, obs, stream=None):
        _check(LIB.heom_observables(self._h, _ptr(y), _ptr(obs), _stream(stream)))

    def tuning(self) -> dict:
        z = _Tuning()
        _check(LIB.heom_get_tuning(self._h, ctypes.byref(z)))
        return {name: getattr(z, name) for name, _ in _Tuning._fields_}

    def set_tuning(self, **kw):
        """Change launch knobs (tile_vars, persistent, xcd_map, max_workgroups,
        spin_limit, cache_policy, transposed, compact). A new tile_vars or a
        change of the transposed copies or compact tiles needs a new upload()
        and new work sizes."""
        cur = self.tuning()
        cur["tile_vars"] = 0
        cur.update(kw)
        z = _Tuning(**cur)
        _check(LIB.heom_set_tuning(self._h, ctypes.byref(z)))

    def max_block(self) -> int:
        """Largest pattern block (unique variables), the smallest allowed tile."""
        lay = self.export_layout()
        n_pat, m = int(lay[0]), int(lay[2])
        pos, best = 4, 0
        for _ in range(n_pat):
            G = int(lay[pos + 1])
            h = 0
            for q in range(G):
                mult = int(lay[pos + 3 + q * (2 + m) + 1])
                h += mult >= 2
            best = max(best, (G + 1) ** 2 + h)
            pos += 3 + G * (2 + m)
        return best

    def work_status(self, work, stream=None):
        """Synchronize and raise HeomError(E_TIMEOUT) if a persistent launch
        that used `work` gave up at a grid barrier."""
        wbytes = work.numel() * work.element_size()
        _check(LIB.heom_work_status(self._h, _ptr(work), wbytes, _stream(stream)))

    def export_layout(self) -> np.ndarray:
        need = ctypes.c_size_t()
        _check(LIB.heom_export_layout(self._h, None, 0, ctypes.byref(need)))
        out = np.zeros(need.value, dtype=np.int64)
        _check(LIB.heom_export_layout(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      need.value, ctypes.byref(need)))
        return out

    def export_coefficients(self) -> np.ndarray:
        need = ctypes.c_size_t()
        _check(LIB.heom_export_coefficients(self._h, None, 0, ctypes.byref(need)))
        out = np.zeros(need.value)
        _check(LIB.heom_export_coefficients(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            need.value, ctypes.byref(need)))
        return out


    def params_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check(LIB.heom_params_bytes(self._h, ctypes.byref(n)))
        return n.value

    def upload_params(self, problem, device_buffer, stream=None):
        """Write the parameter block of `problem` (same structure key) into a
        caller-owned uint8 device buffer."""
        s, keep = _problem_struct(problem)
        nbytes = device_buffer.numel() * device_buffer.element_size()
        _check(LIB.heom_upload_params(self._h, ctypes.byref(s), _ptr(device_buffer), nbytes, _stream(stream)))


class Batch:
    """A set of slots, each an independent problem propagated together."""

    def __init__(self, capacity: int):
        h = ctypes.c_void_p()
        _check(LIB.heom_batch_create(int(capacity), ctypes.byref(h)))
        self._h = h
        self.capacity = capacity
        self._keep = {}      # slot -> objects that must outlive the slot (and its obs stride)
        self._dt = {}        # slot -> time step
        self.image = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and LIB is not None:
            LIB.heom_batch_free(h)
            self._h = None

    def set_slot(self, slot: int, tables: Tables, y, work, dt: float, params=None, obs=None,
                 obs_every: int = 0):
        cap = 0 if obs is None else obs.numel() // HEOM_NOBS
        wbytes = work.numel() * work.element_size()
        _check(LIB.heom_batch_set_slot(self._h, int(slot), tables.handle,
                                       _ptr(params) if params is not None else None, _ptr(y), _ptr(work), wbytes,
                                       float(dt), _ptr(obs) if obs is not None else None, int(obs_every), int(cap)))
        self._keep[slot] = (tables, params, y, work, obs, int(obs_every))
        self._dt[slot] = float(dt)

    def clear_slot(self, slot: int):
        _check(LIB.heom_batch_clear_slot(self._h, int(slot)))
        self._keep.pop(slot, None)
        self._dt.pop(slot, None)

    def device_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check(LIB.heom_batch_device_bytes(self._h, ctypes.byref(n)))
        return n.value

    def commit(self, torch, stream=None):
        """Upload slot records and the tile list into a fresh device buffer."""
        buf = torch.empty(max(self.device_bytes(), 256), dtype=torch.uint8, device="cuda")
        _check(LIB.heom_batch_commit(self._h, _ptr(buf), buf.numel(), _stream(stream)))
        self.image = buf

    def propagate(self, nsteps: int, precision: int = HEOM_FP64, stream=None):
        _check(LIB.heom_batch_propagate(self._h, int(nsteps), int(precision), _stream(stream)))

    def set_graph(self, steps: int):
        """Replay groups of `steps` RK4 steps from a captured HIP graph (0 = off)."""
        _check(LIB.heom_batch_set_graph(self._h, int(steps)))

    def set_merge(self, max_tiles: int):
        """Run the smallest launch groups (m <= 4, at most max_tiles/8 tiles each,
        max_tiles in all) as one launch per stage (0 = one launch per group).
        Takes effect at the next commit."""
        _check(LIB.heom_batch_set_merge(self._h, int(max_tiles)))

    def set_interleave(self, tiles: int):
        """Let the slots of one structure image take turns, `tiles` tiles each,
        in the groups with one workgroup per slot (0 = slot by slot). Takes
        effect at the next commit."""
        _check(LIB.heom_batch_set_interleave(self._h, int(tiles)))

    def status(self, stream=None) -> np.ndarray:
        """Synchronize and return one flag per slot: 1 where the slot's tier-0
        block became NaN or infinite since the last commit (heom_batch_status
        returns E_NONFINITE then; the flags are returned instead of raising)."""
        flags = np.zeros(self.capacity, dtype=np.int32)
        rc = LIB.heom_batch_status(self._h, flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   int(self.capacity), _stream(stream))
        if rc not in (HEOM_OK, -5):
            _check(rc)
        return flags

    def set_share(self, max_slots: int):
        """Compute slots that share one structure image together, up to
        max_slots per workgroup and tile (1 = off). Takes effect at the next
        commit."""
        _check(LIB.heom_batch_set_share(self._h, int(max_slots)))

    def slot_steps(self, slot: int) -> int:
        n = ctypes.c_int64()
        _check(LIB.heom_batch_slot_steps(self._h, int(slot), ctypes.byref(n)))
        return n.value


def reconstruct_work_bytes(N: int) -> int:
    return int(LIB.heom_reconstruct_work_bytes(int(N)))


def reconstruct_dense(N: int, rho0, R: np.ndarray, mask: int, work, out, stream=None):
    """heom_reconstruct_dense: rho0 and out device tensors of (N+1)^2
    complex128, R the HEOM_RECON_R_DOUBLES doubles of the five packed slot
    matrices (host), work a device buffer of reconstruct_work_bytes(N)."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    if R.size != HEOM_RECON_R_DOUBLES:
        raise ValueError(f"R must hold {HEOM_RECON_R_DOUBLES} doubles")
    wbytes = work.numel() * work.element_size()
    _check(LIB.heom_reconstruct_dense(int(N), _ptr(rho0), R.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      int(mask), _ptr(work), wbytes, _ptr(out), _stream(stream)))


def version() -> str:
    return LIB.heom_version().decode()
