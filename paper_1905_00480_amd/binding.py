"""ctypes binding of libsho.so (argument marshalling only).

Every operation runs in the library's gfx950 kernels on the caller's current
torch stream; PyTorch only provides device memory and streams.  There is no
fallback: if the library is missing or no GPU is present the calls raise.

Layouts (see include/sho.h):
  psi   float64 tensor (nz, ny, nx, B) on the GPU, band index fastest
  c, w  float64 tensor with coeff_doubles entries, per-atom blocks
        [N_SHO(nu_a)][B] in atom order (n: nz outer, ny, nx fastest)
  grad  float64 tensor (natoms, 3)
Plans made with FLAG_FP32 take float32 psi and c of the same layouts (an even
number of bands); complex bands are passed as torch.view_as_real views, i.e.
as interleaved (real, imaginary) pairs of 2 x B real bands.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsho.so")

SHO_OK = 0
SHO_E_INVALID = -1
SHO_E_UNDERSAMPLED = -2
SHO_E_NU_RANGE = -3
SHO_E_BOX = -4
SHO_E_NOMEM = -5
SHO_E_DEVICE = -6
SHO_E_BUDGET = -7
SHO_NU_MAX = 10
SHO_SETUP_NU_MAX = 60
FLAG_STORED = 0x1
FLAG_ALLOW_UNDERSAMPLED = 0x2
FLAG_HOST_ONLY = 0x4
FLAG_PER_ATOM = 0x8
FLAG_FP32 = 0x10
FLAG_DETERMINISTIC = 0x20
FLAG_BLOCH = 0x40
SCHED_BY_NU = 0
SCHED_SINGLE = 1
SCHED_SINGLE_LPT = 2
SCHED_SWEEP = 3
PROJECT_ITEMS, PROJECT_BLOCKS = 0, 1
SCHED_XCD = 4
EXPAND_ROWS = 0
EXPAND_BLOCKS = 1
EXPAND_OWNER = 2
SCHEDULES = (SCHED_BY_NU, SCHED_SINGLE, SCHED_SINGLE_LPT, SCHED_SWEEP,
             SCHED_BY_NU | SCHED_XCD, SCHED_SINGLE | SCHED_XCD, SCHED_SINGLE_LPT | SCHED_XCD,
             SCHED_SWEEP | SCHED_XCD)

# every symbol include/sho.h declares
EXPORTS = (
    "sho_nsho", "sho_last_error", "sho_plan_create", "sho_plan_destroy",
    "sho_plan_get_info", "sho_plan_coeff_offsets", "sho_plan_support_counts",
    "sho_plan_set_centres", "sho_plan_project", "sho_plan_expand",
    "sho_plan_project_f32", "sho_plan_expand_f32",
    "sho_plan_force", "sho_project", "sho_expand", "sho_force",
    "sho_plan_expand_scaled", "sho_plan_expand_noalloc", "sho_plan_create_radial",
    "sho_plan_set_kpoint", "sho_plan_set_project", "sho_plan_get_project",
    "sho_plan_set_expand_tile", "sho_plan_get_expand_tile", "sho_plan_tune_expand",
    "sho_cache_clear", "sho_plan_profile", "sho_plan_profile_read",
    "sho_plan_set_schedule", "sho_plan_get_schedule", "sho_plan_tune",
    "sho_plan_set_expand", "sho_plan_get_expand",
    "sho_plan_matrix_offsets", "sho_plan_multiply", "sho_plan_apply",
    "sho_graph_create_apply",
    "sho_graph_create", "sho_graph_launch", "sho_graph_destroy",
    "sho_server_create", "sho_server_add_system", "sho_server_submit",
    "sho_server_drain", "sho_server_request_info", "sho_server_read",
    "sho_plan_release_scratch",
    "sho_server_get_stats", "sho_server_system_info", "sho_server_inputs",
    "sho_server_clock", "sho_server_destroy", "sho_server_prefetch",
    "sho_setup_unitary", "sho_setup_radial", "sho_setup_matrix", "sho_setup_quality",
)
JOB_PROJECT, JOB_EXPAND, JOB_FORCE = 0, 1, 2
KERNEL_KINDS = ("project", "expand_z", "expand_xy", "force")


class ShoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libsho error %d: %s" % (code, msg))
        self.code = code


class sho_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("h", ctypes.c_double),
                ("periodic", ctypes.c_int32 * 3)]


class sho_plan_info(ctypes.Structure):
    _fields_ = [("natoms", ctypes.c_int32), ("nbands", ctypes.c_int32),
                ("nu_max", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("coeff_rows", ctypes.c_int64), ("coeff_doubles", ctypes.c_int64),
                ("support_points", ctypes.c_int64), ("lines", ctypes.c_int64),
                ("planes", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("stored_bytes", ctypes.c_int64), ("union_points", ctypes.c_int64),
                ("expand_points", ctypes.c_int64),
                ("expand_scratch_doubles", ctypes.c_int64),
                ("expand_blocks", ctypes.c_int64), ("expand_entries", ctypes.c_int64)]


class sho_tune_result(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("band_tile", ctypes.c_int32),
                ("target_points", ctypes.c_int64), ("ms", ctypes.c_double),
                ("ms_before", ctypes.c_double), ("candidates", ctypes.c_int32),
                ("project_form", ctypes.c_int32)]


class sho_tune_expand_result(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("band_tile", ctypes.c_int32),
                ("block_rows", ctypes.c_int32), ("block_x", ctypes.c_int32),
                ("ms", ctypes.c_double), ("ms_before", ctypes.c_double),
                ("candidates", ctypes.c_int32), ("pad", ctypes.c_int32)]


class sho_server_stats(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("resident_bytes", ctypes.c_int64),
                ("peak_resident_bytes", ctypes.c_int64), ("requests", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("admissions", ctypes.c_int64),
                ("evictions", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("systems", ctypes.c_int32), ("resident_systems", ctypes.c_int32),
                ("short_requests", ctypes.c_int64), ("plan_reuses", ctypes.c_int64),
                ("plan_drops", ctypes.c_int64)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p


def load_library(path=None):
    """Load libsho.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    import torch  # noqa: F401  -- torch's HIP runtime must be the one in use
    # SHO_LIBRARY names another build of the same library (the host-sanitized
    # libsho_asan.so of `build.py --sanitize`, run with its runtime preloaded)
    p = path or os.environ.get("SHO_LIBRARY") or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            "libsho.so not built: run `python -m paper_1905_00480_amd.build` "
            "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(p)
    G = ctypes.POINTER(sho_grid)
    P = _vp
    lib.sho_nsho.argtypes = [ctypes.c_int32]
    lib.sho_nsho.restype = ctypes.c_int32
    lib.sho_last_error.argtypes = []
    lib.sho_last_error.restype = ctypes.c_char_p
    lib.sho_plan_create.argtypes = [G, ctypes.c_int32, _dp, _dp, _i32p, _dp,
                                    ctypes.c_int32, ctypes.c_uint32,
                                    ctypes.POINTER(_vp)]
    lib.sho_plan_create_radial.argtypes = [G, ctypes.c_int32, _dp, _dp, ctypes.c_int32, _i32p,
                                           ctypes.c_int32, ctypes.c_double, _dp, ctypes.c_int32,
                                           ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)]
    lib.sho_plan_destroy.argtypes = [P]
    lib.sho_plan_release_scratch.argtypes = [P]
    lib.sho_plan_get_info.argtypes = [P, ctypes.POINTER(sho_plan_info)]
    lib.sho_plan_coeff_offsets.argtypes = [P, _i64p]
    lib.sho_plan_support_counts.argtypes = [P, _i64p]
    lib.sho_plan_set_centres.argtypes = [P, _dp, _vp]
    lib.sho_plan_set_kpoint.argtypes = [P, _dp]
    lib.sho_plan_set_project.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32]
    lib.sho_plan_get_project.argtypes = [P, _i32p, _i32p, _i32p, _i32p]
    lib.sho_plan_set_expand_tile.argtypes = [P, ctypes.c_int32]
    lib.sho_plan_get_expand_tile.argtypes = [P, _i32p]
    lib.sho_plan_tune_expand.argtypes = [P, _vp, _vp, ctypes.c_int32, _vp,
                                         ctypes.POINTER(sho_tune_expand_result)]
    lib.sho_plan_project.argtypes = [P, _vp, _vp, _vp]
    lib.sho_plan_expand.argtypes = [P, _vp, _vp, _vp]
    lib.sho_plan_project_f32.argtypes = [P, _vp, _vp, _vp]
    lib.sho_plan_expand_f32.argtypes = [P, _vp, _vp, _vp]
    lib.sho_plan_expand_scaled.argtypes = [P, ctypes.c_double, _vp, _vp, _vp]
    lib.sho_plan_expand_noalloc.argtypes = [P, _vp, _vp, _vp]
    lib.sho_plan_force.argtypes = [P, _vp, _vp, _vp, _vp]
    geo = [G, ctypes.c_int32, _dp, _dp, _i32p, ctypes.c_int32]
    lib.sho_project.argtypes = geo + [_vp, _vp, ctypes.c_uint32, _vp]
    lib.sho_expand.argtypes = geo + [_vp, _vp, ctypes.c_uint32, _vp]
    lib.sho_force.argtypes = geo + [_vp, _vp, _vp, ctypes.c_uint32, _vp]
    lib.sho_cache_clear.argtypes = []
    lib.sho_plan_profile.argtypes = [P, ctypes.c_int32]
    lib.sho_plan_profile_read.argtypes = [P, _i64p, _dp]
    lib.sho_plan_set_schedule.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]
    lib.sho_plan_get_schedule.argtypes = [P, _i32p, _i32p, _i64p]
    lib.sho_plan_set_expand.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.sho_plan_get_expand.argtypes = [P, _i32p, _i32p, _i32p]
    lib.sho_plan_tune.argtypes = [P, _vp, _vp, ctypes.c_int32, _vp,
                                  ctypes.POINTER(sho_tune_result)]
    lib.sho_graph_create.argtypes = [P, _vp, _vp, _vp, ctypes.POINTER(_vp)]
    lib.sho_graph_launch.argtypes = [_vp, _vp]
    lib.sho_plan_matrix_offsets.argtypes = [P, _i64p]
    lib.sho_plan_multiply.argtypes = [P, _vp, _vp, _vp, _vp]
    lib.sho_plan_apply.argtypes = [P, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.sho_graph_create_apply.argtypes = [P, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]
    lib.sho_graph_destroy.argtypes = [_vp]
    lib.sho_server_create.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                      ctypes.POINTER(_vp)]
    lib.sho_server_add_system.argtypes = [P, G, ctypes.c_int32, _dp, _dp, _i32p,
                                          ctypes.c_int32, _dp, _dp, _i32p]
    lib.sho_server_submit.argtypes = [P, ctypes.c_int32, ctypes.c_int32, _i64p]
    lib.sho_server_drain.argtypes = [P]
    lib.sho_server_prefetch.argtypes = [P, ctypes.c_int32]
    lib.sho_server_request_info.argtypes = [P, ctypes.c_int64, _i32p, _i32p, _dp, _dp]
    lib.sho_server_read.argtypes = [P, ctypes.c_int32, ctypes.c_int32, _dp]
    lib.sho_server_get_stats.argtypes = [P, ctypes.POINTER(sho_server_stats)]
    lib.sho_server_system_info.argtypes = [P, ctypes.c_int32, _i64p, _i32p]
    lib.sho_server_inputs.argtypes = [P, ctypes.c_int32, ctypes.POINTER(_dp),
                                      ctypes.POINTER(_dp)]
    lib.sho_server_clock.argtypes = [P, _dp]
    lib.sho_server_destroy.argtypes = [P]
    lib.sho_setup_unitary.argtypes = [ctypes.c_int32, _dp]
    lib.sho_setup_radial.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int64, _dp, _dp]
    lib.sho_setup_matrix.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _i32p,
                                     ctypes.c_int64, _dp, _dp, _dp, _dp, _dp]
    lib.sho_setup_quality.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                      ctypes.c_int64, _dp, _dp, _dp, _dp]
    for name in EXPORTS:
        if name not in ("sho_nsho", "sho_last_error"):
            getattr(lib, name).restype = ctypes.c_int32
    if path is None:
        _lib = lib
    return lib


def _check(code):
    if code != SHO_OK:
        msg = load_library().sho_last_error().decode(errors="replace")
        raise ShoError(code, msg)


def make_grid(n, h, periodic):
    g = sho_grid()
    for d in range(3):
        g.n[d] = int(n[d])
        g.periodic[d] = 1 if periodic[d] else 0
    g.h = float(h)
    return g


def _host_f64(a, shape):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))


def _host_i32(a, shape):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(shape))


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, numel, name, f32=False):
    """Device pointer of a contiguous GPU tensor of `numel` real elements
    (complex tensors count their real and imaginary parts)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a GPU tensor" % name)
    if t.is_complex():
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        t = torch.view_as_real(t)
    want = torch.float32 if f32 else torch.float64
    if t.dtype != want:
        raise TypeError("%s must be %s" % (name, str(want).split(".")[-1]))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Reusable geometry plan: supports, line tables, device buffers."""

    def __init__(self, n, h, periodic, pos, sigma, numax, nbands, rbox=None,
                 flags=0):
        lib = load_library()
        self._lib = lib
        self.n = tuple(int(v) for v in n)
        self.h = float(h)
        self.periodic = tuple(bool(v) for v in periodic)
        pos = _host_f64(pos, (-1, 3))
        self.natoms = pos.shape[0]
        self._pos = pos
        self._centres = pos.copy()  # the function centres the plan holds now
        self._sigma = _host_f64(sigma, (self.natoms,))
        self._numax = _host_i32(numax, (self.natoms,))
        self._rbox = None if rbox is None else _host_f64(rbox, (self.natoms,))
        self.nbands = int(nbands)
        self._grid = make_grid(self.n, self.h, self.periodic)
        handle = ctypes.c_void_p()
        _check(lib.sho_plan_create(
            ctypes.byref(self._grid), self.natoms,
            self._pos.ctypes.data_as(_dp), self._sigma.ctypes.data_as(_dp),
            self._numax.ctypes.data_as(_i32p),
            None if self._rbox is None else self._rbox.ctypes.data_as(_dp),
            self.nbands, int(flags), ctypes.byref(handle)))
        self._adopt(handle, flags)

    def _adopt(self, handle, flags):
        self._h = handle
        self.fp32 = bool(int(flags) & FLAG_FP32)
        self.bloch = bool(int(flags) & FLAG_BLOCH)
        info = sho_plan_info()
        _check(self._lib.sho_plan_get_info(self._h, ctypes.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in sho_plan_info._fields_}
        self.coeff_doubles = int(info.coeff_doubles)
        self.support_points = int(info.support_points)

    @classmethod
    def radial(cls, n, h, periodic, pos, rcut, ell, dr, tables, nbands, flags=0):
        """Plan over stored numerical projectors P_k(r) Y_lm (sho_plan_create_radial):
        ell [nradial], tables [nradial][nr] on the radial grid i*dr, rcut [natoms]."""
        self = cls.__new__(cls)
        lib = load_library()
        self._lib = lib
        self.n = tuple(int(v) for v in n)
        self.h = float(h)
        self.periodic = tuple(bool(v) for v in periodic)
        pos = _host_f64(pos, (-1, 3))
        self.natoms = pos.shape[0]
        self._pos = pos
        self._centres = pos.copy()
        self._rcut = _host_f64(rcut, (self.natoms,))
        self._ell = _host_i32(ell, (-1,))
        tables = _host_f64(tables, (self._ell.size, -1))
        self._tables = tables
        self.nbands = int(nbands)
        self._grid = make_grid(self.n, self.h, self.periodic)
        handle = ctypes.c_void_p()
        _check(lib.sho_plan_create_radial(
            ctypes.byref(self._grid), self.natoms, self._pos.ctypes.data_as(_dp),
            self._rcut.ctypes.data_as(_dp), int(self._ell.size),
            self._ell.ctypes.data_as(_i32p), int(tables.shape[1]), float(dr),
            tables.ctypes.data_as(_dp), self.nbands, int(flags), ctypes.byref(handle)))
        self._adopt(handle, flags)
        return self

    @classmethod
    def from_system(cls, s, flags=0, rbox=None):
        return cls(s.n, s.h, s.periodic, s.pos, s.sigma, s.numax, s.nbands,
                   rbox=rbox if rbox is not None else s.rbox, flags=flags)

    @property
    def psi_numel(self):
        """Real elements of psi (complex bands of Bloch plans count twice)."""
        return self.n[0] * self.n[1] * self.n[2] * self.nbands * (2 if self.bloch else 1)

    def set_kpoint(self, k):
        """Bloch wave vector (Bohr^-1) of a FLAG_BLOCH plan."""
        k = _host_f64(k, (3,))
        _check(self._lib.sho_plan_set_kpoint(self._h, k.ctypes.data_as(_dp)))

    def coeff_offsets(self):
        off = np.empty(self.natoms + 1, dtype=np.int64)
        _check(self._lib.sho_plan_coeff_offsets(self._h, off.ctypes.data_as(_i64p)))
        return off

    def support_counts(self):
        cnt = np.empty(max(self.natoms, 1), dtype=np.int64)
        _check(self._lib.sho_plan_support_counts(self._h, cnt.ctypes.data_as(_i64p)))
        return cnt[:self.natoms]

    def set_centres(self, pos, stream=None):
        pos = _host_f64(pos, (self.natoms, 3))
        _check(self._lib.sho_plan_set_centres(self._h, pos.ctypes.data_as(_dp),
                                              _stream(stream)))
        self._centres = pos.copy()

    def centres(self):
        """The function centres the plan holds (host copy)."""
        return self._centres.copy()

    def project(self, psi, c=None, stream=None):
        import torch
        f32 = self.fp32
        if c is None:
            if self.bloch:
                c = torch.empty(self.coeff_doubles // 2,
                                dtype=torch.complex64 if f32 else torch.complex128,
                                device=psi.device)
            else:
                c = torch.empty(self.coeff_doubles,
                                dtype=torch.float32 if f32 else torch.float64, device=psi.device)
        fn = self._lib.sho_plan_project_f32 if f32 else self._lib.sho_plan_project
        _check(fn(self._h, _dev(psi, self.psi_numel, "psi", f32),
                  _dev(c, self.coeff_doubles, "c", f32), _stream(stream)))
        return c

    def expand(self, c, psi, stream=None, alpha=None):
        """psi += expansion of c (times alpha, if given: FP64 plans)."""
        f32 = self.fp32
        if alpha is not None:
            _check(self._lib.sho_plan_expand_scaled(
                self._h, float(alpha), _dev(c, self.coeff_doubles, "c"),
                _dev(psi, self.psi_numel, "psi"), _stream(stream)))
            return psi
        fn = self._lib.sho_plan_expand_f32 if f32 else self._lib.sho_plan_expand
        _check(fn(self._h, _dev(c, self.coeff_doubles, "c", f32),
                  _dev(psi, self.psi_numel, "psi", f32), _stream(stream)))
        return psi

    def expand_noalloc(self, c, psi, stream=None):
        """psi += expansion of c with the library's static scratch (FP64 plans;
        allocates nothing; calls overlapping on one device race)."""
        _check(self._lib.sho_plan_expand_noalloc(
            self._h, _dev(c, self.coeff_doubles, "c"), _dev(psi, self.psi_numel, "psi"),
            _stream(stream)))
        return psi

    def force(self, psi, w, grad=None, stream=None):
        import torch
        if grad is None:
            grad = torch.empty((self.natoms, 3), dtype=torch.float64, device=psi.device)
        _check(self._lib.sho_plan_force(
            self._h, _dev(psi, self.psi_numel, "psi"),
            _dev(w, self.coeff_doubles, "w"), _dev(grad, 3 * self.natoms, "grad"),
            _stream(stream)))
        return grad

    def matrix_offsets(self):
        """Per-atom offsets (doubles) of the atomic matrices in D."""
        off = np.empty(self.natoms + 1, dtype=np.int64)
        _check(self._lib.sho_plan_matrix_offsets(self._h, off.ctypes.data_as(_i64p)))
        return off

    def multiply(self, D, c, d=None, stream=None):
        """d[a] = D_a c[a] for every atom."""
        import torch
        if d is None:
            d = torch.empty_like(c)
        nD = int(self.matrix_offsets()[-1])
        _check(self._lib.sho_plan_multiply(self._h, _dev(D, nD, "D"),
                                           _dev(c, self.coeff_doubles, "c"),
                                           _dev(d, self.coeff_doubles, "d"), _stream(stream)))
        return d

    def apply(self, psi, D, out, c=None, d=None, stream=None):
        """out += sum_a P_a D_a P_a^T psi (with h^3 in the projection)."""
        import torch
        if c is None:
            c = torch.empty(self.coeff_doubles, dtype=torch.float64, device=psi.device)
        if d is None:
            d = torch.empty_like(c)
        nD = int(self.matrix_offsets()[-1])
        _check(self._lib.sho_plan_apply(
            self._h, _dev(psi, self.psi_numel, "psi"), _dev(D, nD, "D"),
            _dev(c, self.coeff_doubles, "c"), _dev(d, self.coeff_doubles, "d"),
            _dev(out, self.psi_numel, "out"), _stream(stream)))
        return out

    def apply_graph(self, psi, D, c, d, out):
        """A replayable graph of apply (project, multiply, expand)."""
        return Graph(self, psi, c, out, D=D, d=d)

    def set_schedule(self, schedule, band_tile=0, target_points=16384):
        _check(self._lib.sho_plan_set_schedule(self._h, int(schedule), int(band_tile),
                                               int(target_points)))

    def schedule(self):
        """(schedule, band_tile, target_points) of the projection."""
        sc, bt, tp = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(self._lib.sho_plan_get_schedule(self._h, ctypes.byref(sc), ctypes.byref(bt),
                                               ctypes.byref(tp)))
        return sc.value, bt.value, tp.value

    def set_project(self, form, block_rows=0, block_x=0, band_tile=0):
        """Projection form: PROJECT_ITEMS or PROJECT_BLOCKS (with block shape and
        band tile; 0 picks the default)."""
        _check(self._lib.sho_plan_set_project(self._h, int(form), int(block_rows),
                                              int(block_x), int(band_tile)))

    def project_form(self):
        """(form, block_rows, block_x, band_tile) of the projection."""
        v = [ctypes.c_int32() for _ in range(4)]
        _check(self._lib.sho_plan_get_project(self._h, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def set_expand(self, mode, block_rows=0, block_x=0):
        """Expansion form: EXPAND_ROWS, EXPAND_BLOCKS or EXPAND_OWNER (with
        block shape; 0 picks the default)."""
        _check(self._lib.sho_plan_set_expand(self._h, int(mode), int(block_rows),
                                             int(block_x)))

    def expand_form(self):
        """(mode, block_rows, block_x) of the expansion."""
        m, r, x = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.sho_plan_get_expand(self._h, ctypes.byref(m), ctypes.byref(r),
                                             ctypes.byref(x)))
        return m.value, r.value, x.value

    def set_expand_tile(self, band_tile):
        """Band tile of the expansion's block form (8..64, 0: default)."""
        _check(self._lib.sho_plan_set_expand_tile(self._h, int(band_tile)))

    def expand_tile(self):
        v = ctypes.c_int32()
        _check(self._lib.sho_plan_get_expand_tile(self._h, ctypes.byref(v)))
        return v.value

    def tune_expand(self, c, psi_scratch, reps=3, stream=None):
        """Time the expansion forms on c -> psi_scratch (its contents are
        overwritten by accumulations) and keep the fastest."""
        r = sho_tune_expand_result()
        _check(self._lib.sho_plan_tune_expand(
            self._h, _dev(c, self.coeff_doubles, "c", self.fp32),
            _dev(psi_scratch, self.psi_numel, "psi", self.fp32),
            int(reps), _stream(stream), ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in sho_tune_expand_result._fields_ if k != "pad"}

    def tune(self, psi, c, reps=3, stream=None):
        """Time the projection schedules on psi -> c and keep the fastest."""
        r = sho_tune_result()
        _check(self._lib.sho_plan_tune(
            self._h, _dev(psi, self.psi_numel, "psi", self.fp32),
            _dev(c, self.coeff_doubles, "c", self.fp32),
            int(reps), _stream(stream), ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in sho_tune_result._fields_}

    def graph(self, psi, c, out):
        """A replayable graph of project(psi -> c) then expand(c -> out)."""
        return Graph(self, psi, c, out)

    def profile(self, enable=True):
        """Start (clear) or stop per-kernel event timing of this plan."""
        _check(self._lib.sho_plan_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """{kind: (launches, mean ms)} of the calls made while profiling."""
        cnt = np.zeros(len(KERNEL_KINDS), dtype=np.int64)
        ms = np.zeros(len(KERNEL_KINDS))
        _check(self._lib.sho_plan_profile_read(self._h, cnt.ctypes.data_as(_i64p),
                                               ms.ctypes.data_as(_dp)))
        return {k: (int(cnt[i]), float(ms[i])) for i, k in enumerate(KERNEL_KINDS)}

    def release_scratch(self):
        """Free the plan's device scratch (plane partials); kept tables."""
        _check(self._lib.sho_plan_release_scratch(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(self._lib.sho_plan_destroy(self._h))
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """Captured project -> expand of a plan on fixed buffers (sho_graph_*).
    Holds references to the plan and the buffers so that they outlive it."""

    def __init__(self, plan, psi, c, out, D=None, d=None):
        self._lib = plan._lib
        self._keep = (plan, psi, c, out, D, d)
        h = ctypes.c_void_p()
        if D is None:
            _check(self._lib.sho_graph_create(
                plan._h, _dev(psi, plan.psi_numel, "psi"), _dev(c, plan.coeff_doubles, "c"),
                _dev(out, plan.psi_numel, "out"), ctypes.byref(h)))
        else:
            nD = int(plan.matrix_offsets()[-1])
            _check(self._lib.sho_graph_create_apply(
                plan._h, _dev(psi, plan.psi_numel, "psi"), _dev(D, nD, "D"),
                _dev(c, plan.coeff_doubles, "c"), _dev(d, plan.coeff_doubles, "d"),
                _dev(out, plan.psi_numel, "out"), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(self._lib.sho_graph_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(self._lib.sho_graph_destroy(self._h))
        self._h = ctypes.c_void_p()
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request server over resident systems (sho_server_*).  Systems are
    workloads.System-like objects (n, h, periodic, pos, sigma, numax,
    nbands)."""

    def __init__(self, budget_bytes, nstreams=4, flags=0):
        self._lib = load_library()
        h = ctypes.c_void_p()
        _check(self._lib.sho_server_create(int(budget_bytes), int(nstreams), int(flags),
                                           ctypes.byref(h)))
        self._h = h
        self._shapes = []

    def add(self, s, psi=None, w=None):
        """Register a system; psi / w (host arrays) are copied, or left zero
        for filling in place through inputs()."""
        grid = make_grid(s.n, s.h, s.periodic)
        pos = _host_f64(s.pos, (-1, 3))
        na = pos.shape[0]
        sig = _host_f64(s.sigma, (na,))
        nu = _host_i32(s.numax, (na,))
        ncoef = _ncoeff(nu, s.nbands)
        npsi = int(np.prod(s.n)) * int(s.nbands)
        pp = None if psi is None else _host_f64(psi, (npsi,))
        ww = None if w is None else _host_f64(w, (ncoef,))
        sid = ctypes.c_int32()
        _check(self._lib.sho_server_add_system(
            self._h, ctypes.byref(grid), na, pos.ctypes.data_as(_dp), sig.ctypes.data_as(_dp),
            nu.ctypes.data_as(_i32p), int(s.nbands),
            None if pp is None else pp.ctypes.data_as(_dp),
            None if ww is None else ww.ctypes.data_as(_dp), ctypes.byref(sid)))
        self._shapes.append((npsi, ncoef, na))
        return sid.value

    def inputs(self, sid):
        """numpy views of the system's pinned psi and w input buffers."""
        pp, ww = _dp(), _dp()
        _check(self._lib.sho_server_inputs(self._h, int(sid), ctypes.byref(pp),
                                           ctypes.byref(ww)))
        npsi, ncoef, _ = self._shapes[sid]
        if not pp:
            return None, None
        return (np.ctypeslib.as_array(pp, shape=(npsi,)),
                np.ctypeslib.as_array(ww, shape=(max(ncoef, 1),))[:ncoef])

    def submit(self, sid, job):
        rid = ctypes.c_int64()
        _check(self._lib.sho_server_submit(self._h, int(sid), int(job), ctypes.byref(rid)))
        return rid.value

    def drain(self):
        _check(self._lib.sho_server_drain(self._h))

    def prefetch(self, sid):
        """Make the system resident now (waits for its upload)."""
        _check(self._lib.sho_server_prefetch(self._h, int(sid)))

    def clock(self):
        t = ctypes.c_double()
        _check(self._lib.sho_server_clock(self._h, ctypes.byref(t)))
        return t.value

    def request_info(self, rid):
        sy, jb = ctypes.c_int32(), ctypes.c_int32()
        ts, td = ctypes.c_double(), ctypes.c_double()
        _check(self._lib.sho_server_request_info(self._h, int(rid), ctypes.byref(sy),
                                                 ctypes.byref(jb), ctypes.byref(ts),
                                                 ctypes.byref(td)))
        return sy.value, jb.value, ts.value, td.value

    def read(self, sid, job):
        npsi, ncoef, na = self._shapes[sid]
        n = {JOB_PROJECT: ncoef, JOB_EXPAND: npsi, JOB_FORCE: 3 * na}[job]
        out = np.empty(max(n, 1))
        _check(self._lib.sho_server_read(self._h, int(sid), int(job), out.ctypes.data_as(_dp)))
        return out[:n]

    def stats(self):
        st = sho_server_stats()
        _check(self._lib.sho_server_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in sho_server_stats._fields_}

    def system_info(self, sid):
        ch, rs = ctypes.c_int64(), ctypes.c_int32()
        _check(self._lib.sho_server_system_info(self._h, int(sid), ctypes.byref(ch),
                                                ctypes.byref(rs)))
        return ch.value, bool(rs.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(self._lib.sho_server_destroy(self._h))
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _geo(n, h, periodic, pos, sigma, numax):
    pos = _host_f64(pos, (-1, 3))
    na = pos.shape[0]
    return (make_grid(n, h, periodic), na, pos, _host_f64(sigma, (na,)),
            _host_i32(numax, (na,)))


def _ncoeff(numax, nbands):
    nu = np.asarray(numax, dtype=np.int64)
    return int(((nu + 1) * (nu + 2) * (nu + 3) // 6).sum()) * int(nbands)


def project(n, h, periodic, pos, sigma, numax, psi, c=None, flags=0, stream=None):
    """Stateless projection (plan built or reused from the library's cache)."""
    import torch
    lib = load_library()
    g, na, pos, sigma, numax = _geo(n, h, periodic, pos, sigma, numax)
    B = psi.shape[-1]
    if c is None:
        c = torch.empty(_ncoeff(numax, B), dtype=torch.float64, device=psi.device)
    _check(lib.sho_project(ctypes.byref(g), na, pos.ctypes.data_as(_dp),
                           sigma.ctypes.data_as(_dp), numax.ctypes.data_as(_i32p), B,
                           _dev(psi, psi.numel(), "psi"),
                           _dev(c, _ncoeff(numax, B), "c"), int(flags), _stream(stream)))
    return c


def expand(n, h, periodic, pos, sigma, numax, c, psi, flags=0, stream=None):
    lib = load_library()
    g, na, pos, sigma, numax = _geo(n, h, periodic, pos, sigma, numax)
    B = psi.shape[-1]
    _check(lib.sho_expand(ctypes.byref(g), na, pos.ctypes.data_as(_dp),
                          sigma.ctypes.data_as(_dp), numax.ctypes.data_as(_i32p), B,
                          _dev(c, _ncoeff(numax, B), "c"),
                          _dev(psi, psi.numel(), "psi"), int(flags), _stream(stream)))
    return psi


def force(n, h, periodic, pos, sigma, numax, psi, w, grad=None, flags=0, stream=None):
    import torch
    lib = load_library()
    g, na, pos, sigma, numax = _geo(n, h, periodic, pos, sigma, numax)
    B = psi.shape[-1]
    if grad is None:
        grad = torch.empty((na, 3), dtype=torch.float64, device=psi.device)
    _check(lib.sho_force(ctypes.byref(g), na, pos.ctypes.data_as(_dp),
                         sigma.ctypes.data_as(_dp), numax.ctypes.data_as(_i32p), B,
                         _dev(psi, psi.numel(), "psi"), _dev(w, _ncoeff(numax, B), "w"),
                         _dev(grad, 3 * na, "grad"), int(flags), _stream(stream)))
    return grad


def nsho(nu):
    return load_library().sho_nsho(int(nu))


def cache_clear():
    _check(load_library().sho_cache_clear())


# ------------------------------------------------------------ set-up side --

def _nsho(nu):
    return (nu + 1) * (nu + 2) * (nu + 3) // 6


def setup_unitary(nu_max):
    """U[c][s] = <Phi_c | Psi_s> (rows: coefficient order, columns: radial order)."""
    lib = load_library()
    N = _nsho(int(nu_max))
    U = np.empty((N, N))
    _check(lib.sho_setup_unitary(int(nu_max), U.ctypes.data_as(_dp)))
    return U


def setup_radial(nu_max, sigma, r):
    """R[k][i] = R_{nr l}(r_i; sigma), k over (nu ascending, l ascending)."""
    lib = load_library()
    r = _host_f64(r, (-1,))
    count = sum(len(range(nu % 2, nu + 1, 2)) for nu in range(int(nu_max) + 1))
    R = np.empty((count, r.size))
    _check(lib.sho_setup_radial(int(nu_max), float(sigma), r.size, r.ctypes.data_as(_dp),
                                R.ctypes.data_as(_dp)))
    return R


def setup_matrix(nu_max, sigma, ell, r, w, P, D):
    """The atomic matrix D of projectors P_k(r) Y_lm in the Cartesian SHO basis."""
    lib = load_library()
    ell = _host_i32(ell, (-1,))
    r = _host_f64(r, (-1,))
    w = _host_f64(w, (r.size,))
    P = _host_f64(P, (ell.size, r.size))
    D = _host_f64(D, (-1,))
    if np.all(ell >= 0):  # (a negative l is left to the library to refuse)
        nproj = int(np.sum(2 * ell + 1))
        if D.size != nproj * nproj:
            raise ValueError("D must be [%d][%d]" % (nproj, nproj))
    N = _nsho(int(nu_max))
    out = np.empty((N, N))
    _check(lib.sho_setup_matrix(int(nu_max), float(sigma), ell.size, ell.ctypes.data_as(_i32p),
                                r.size, r.ctypes.data_as(_dp), w.ctypes.data_as(_dp),
                                P.ctypes.data_as(_dp), D.ctypes.data_as(_dp),
                                out.ctypes.data_as(_dp)))
    return out


def setup_quality(nu_max, sigma, ell, r, w, P):
    """Q[nu], nu = 0..nu_max, of one radial projector (sec. 4)."""
    lib = load_library()
    r = _host_f64(r, (-1,))
    w = _host_f64(w, (r.size,))
    P = _host_f64(P, (r.size,))
    Q = np.empty(int(nu_max) + 1)
    _check(lib.sho_setup_quality(int(nu_max), float(sigma), int(ell), r.size,
                                 r.ctypes.data_as(_dp), w.ctypes.data_as(_dp),
                                 P.ctypes.data_as(_dp), Q.ctypes.data_as(_dp)))
    return Q
