"""Thin Python binding of the C ABI in include/mjk.h (argument marshalling only).

Every step of the ERI / J-K path runs in the HIP library
paper_2412_13203_amd/_lib/libmjk.so; torch provides device memory and the
stream.  There is no fallback: if the library or a gfx950 device is missing,
calls raise.

    plan = Plan(basis, tau=1e-10)          # mjk_plan_create + mjk_plan_bind
    J, K = plan.build_jk(D)                # mjk_build_jk
    blocks = plan.eri_class(quartets)      # mjk_eri_class
    e = E2.apply(coords, D, basis)         # mjk_build_jk + mjk_e2; backward: mjk_grad_e2
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MJK_LIBRARY selects another build of the same library (A/B measurements)
LIB_PATH = os.environ.get("MJK_LIBRARY") or os.path.join(_HERE, "_lib", "libmjk.so")

MJK_OK = 0
ERRORS = {-1: "MJK_ERR_INVALID_ARG", -2: "MJK_ERR_UNSUPPORTED", -3: "MJK_ERR_NO_DEVICE", -4: "MJK_ERR_WORKSPACE",
          -5: "MJK_ERR_HIP", -6: "MJK_ERR_STATE"}
FLAG_CHECK = 0x1
FLAG_GRAD = 0x2
FLAG_NO_STAGING = 0x4
FLAG_PERSISTENT = 0x8
FLAG_NO_KBINS = 0x10


class MjkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Basis(ctypes.Structure):
    _fields_ = [
        ("natom", ctypes.c_int32),
        ("xyz", ctypes.POINTER(ctypes.c_double)),
        ("nshell", ctypes.c_int32),
        ("shell_atom", ctypes.POINTER(ctypes.c_int32)),
        ("shell_l", ctypes.POINTER(ctypes.c_int32)),
        ("shell_nprim", ctypes.POINTER(ctypes.c_int32)),
        ("shell_prim_off", ctypes.POINTER(ctypes.c_int32)),
        ("nprim", ctypes.c_int64),
        ("exps", ctypes.POINTER(ctypes.c_double)),
        ("coefs", ctypes.POINTER(ctypes.c_double)),
    ]


class JKOpts(ctypes.Structure):
    _fields_ = [("schwarz_tau", ctypes.c_double), ("fp32_tau", ctypes.c_double), ("flags", ctypes.c_uint32)]


class PlanStats(ctypes.Structure):
    _fields_ = [
        ("nbf", ctypes.c_int64), ("nshell", ctypes.c_int64), ("npair", ctypes.c_int64),
        ("nprim_pair", ctypes.c_int64), ("nquartet_total", ctypes.c_int64), ("nquartet_kept", ctypes.c_int64),
        ("nquartet_fp32", ctypes.c_int64),
        ("nprim_quartet_kept", ctypes.c_int64), ("ncart_eri_kept", ctypes.c_int64), ("nlaunch", ctypes.c_int64),
        ("vrr_flops_kept", ctypes.c_double), ("workspace_bytes", ctypes.c_size_t),
        ("grad_flops_kept", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ClassTiming(ctypes.Structure):
    _fields_ = [("la", ctypes.c_int32), ("lb", ctypes.c_int32), ("lc", ctypes.c_int32), ("ld", ctypes.c_int32),
                ("nlaunch", ctypes.c_int32), ("ms", ctypes.c_double), ("nquartet", ctypes.c_int64),
                ("nprim_quartet", ctypes.c_int64), ("flops", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["cls"] = "".join("spdf"[d[k]] for k in ("la", "lb", "lc", "ld"))
        return d


_lib = None

# exported names of include/mjk.h
EXPORTS = ["mjk_lmax", "mjk_grad_lmax", "mjk_num_classes", "mjk_class_l", "mjk_last_error", "mjk_ctx_last_error",
           "mjk_ctx_create", "mjk_ctx_destroy", "mjk_boys",
           "mjk_nbf", "mjk_plan_create", "mjk_plan_bind", "mjk_plan_set_tiles", "mjk_build_jk", "mjk_build_jk_static", "mjk_e2",
           "mjk_grad_e2", "mjk_e2_backward", "mjk_eri_class", "mjk_schwarz", "mjk_one_electron", "mjk_num_kbuckets",
           "mjk_plan_set_density_screen", "mjk_plan_stats_get", "mjk_plan_set_timing",
           "mjk_plan_timings", "mjk_plan_destroy",
           "mjk_batch_create", "mjk_batch_bind", "mjk_batch_offsets", "mjk_batch_build_jk", "mjk_batch_set_tiles",
           "mjk_batch_autotune", "mjk_batch_set_stamps", "mjk_batch_mol_times", "mjk_batch_set_timing",
           "mjk_batch_timings", "mjk_batch_stats", "mjk_batch_destroy"]


def lib():
    """Load libmjk.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MjkError(-3, f"{LIB_PATH} is missing: run `python -m paper_2412_13203_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.mjk_lmax.restype = ctypes.c_int
        L.mjk_grad_lmax.restype = ctypes.c_int
        L.mjk_ctx_last_error.argtypes = [vp]
        L.mjk_ctx_last_error.restype = ctypes.c_char_p
        L.mjk_boys.argtypes = [vp, i32, vp, i64, vp, vp]
        L.mjk_e2_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.mjk_num_classes.restype = ctypes.c_int
        L.mjk_num_kbuckets.restype = ctypes.c_int
        L.mjk_class_l.argtypes = [i32, ctypes.POINTER(i32)]
        L.mjk_plan_set_tiles.argtypes = [vp, ctypes.POINTER(i32), i32]
        L.mjk_batch_create.argtypes = [vp, i32, ctypes.POINTER(Basis), ctypes.POINTER(JKOpts), ctypes.POINTER(vp),
                                       ctypes.POINTER(sz)]
        L.mjk_batch_bind.argtypes = [vp, vp, sz, vp]
        L.mjk_batch_offsets.argtypes = [vp, ctypes.POINTER(i64)]
        L.mjk_batch_build_jk.argtypes = [vp, vp, vp, vp, vp]
        L.mjk_batch_set_tiles.argtypes = [vp, ctypes.POINTER(i32), i32]
        L.mjk_batch_autotune.argtypes = [vp, vp, vp, vp, i32, ctypes.POINTER(i32), i32, vp]
        L.mjk_batch_set_stamps.argtypes = [vp, ctypes.c_int]
        L.mjk_batch_mol_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.mjk_batch_set_timing.argtypes = [vp, ctypes.c_int]
        L.mjk_batch_timings.argtypes = [vp, ctypes.POINTER(ClassTiming), i32, ctypes.POINTER(i32)]
        L.mjk_batch_stats.argtypes = [vp, ctypes.POINTER(PlanStats), ctypes.POINTER(i64)]
        L.mjk_batch_destroy.argtypes = [vp]
        L.mjk_batch_destroy.restype = None
        L.mjk_last_error.restype = ctypes.c_char_p
        L.mjk_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
        L.mjk_ctx_destroy.argtypes = [vp]
        L.mjk_ctx_destroy.restype = None
        L.mjk_nbf.argtypes = [ctypes.POINTER(Basis), ctypes.POINTER(i64)]
        L.mjk_plan_create.argtypes = [vp, ctypes.POINTER(Basis), ctypes.POINTER(JKOpts), ctypes.POINTER(vp),
                                      ctypes.POINTER(sz)]
        L.mjk_plan_bind.argtypes = [vp, vp, sz, vp]
        L.mjk_build_jk.argtypes = [vp, vp, vp, vp, vp]
        L.mjk_build_jk_static.argtypes = [vp, vp, vp, vp, vp]
        L.mjk_e2.argtypes = [vp, vp, vp, vp, vp, vp]
        L.mjk_grad_e2.argtypes = [vp, vp, vp, vp]
        L.mjk_eri_class.argtypes = [vp, ctypes.POINTER(i32), i64, vp, i64, vp]
        L.mjk_schwarz.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.mjk_one_electron.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.mjk_plan_set_density_screen.argtypes = [vp, vp, ctypes.c_double, vp]
        L.mjk_plan_stats_get.argtypes = [vp, ctypes.POINTER(PlanStats)]
        L.mjk_plan_set_timing.argtypes = [vp, ctypes.c_int]
        L.mjk_plan_timings.argtypes = [vp, ctypes.POINTER(ClassTiming), i32, ctypes.POINTER(i32)]
        L.mjk_plan_destroy.argtypes = [vp]
        L.mjk_plan_destroy.restype = None
        _lib = L
    return _lib


def _cache_read(path: str) -> dict:
    """Autotune tables stored at `path` ({} if the file does not exist)."""
    try:
        with open(path) as fh:
            return json.load(fh)
    except FileNotFoundError:
        return {}


def _check(rc):
    if rc != MJK_OK:
        raise MjkError(rc, lib().mjk_last_error().decode())


class _HostBasis:
    """Contiguous host arrays + the mjk_basis struct that points at them."""

    def __init__(self, basis: dict):
        self.xyz = np.ascontiguousarray(basis["xyz"], dtype=np.float64)
        self.atom = np.ascontiguousarray(basis["shell_atom"], dtype=np.int32)
        self.l = np.ascontiguousarray(basis["shell_l"], dtype=np.int32)
        self.nprim = np.ascontiguousarray(basis["shell_nprim"], dtype=np.int32)
        self.off = np.ascontiguousarray(basis["shell_prim_off"], dtype=np.int32)
        self.exps = np.ascontiguousarray(basis["exps"], dtype=np.float64)
        self.coefs = np.ascontiguousarray(basis["coefs"], dtype=np.float64)
        d = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
        i = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))  # noqa: E731
        self.s = Basis(self.xyz.shape[0], d(self.xyz), len(self.l), i(self.atom), i(self.l), i(self.nprim),
                       i(self.off), len(self.exps), d(self.exps), d(self.coefs))
        self.ncart = (self.l + 1) * (self.l + 2) // 2


def nbf(basis: dict) -> int:
    h = _HostBasis(basis)
    n = ctypes.c_int64(0)
    _check(lib().mjk_nbf(ctypes.byref(h.s), ctypes.byref(n)))
    return int(n.value)


_ctx = {}


def context(device: int = 0):
    if device not in _ctx:
        c = ctypes.c_void_p()
        _check(lib().mjk_ctx_create(device, ctypes.byref(c)))
        _ctx[device] = c
    return _ctx[device]


def _stream(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def context_last_error(device: int = 0) -> str:
    """Message of the last failed call made with the device's context."""
    return lib().mjk_ctx_last_error(context(device)).decode()


def boys(T, mmax: int, device: int = 0):
    """F_m(T), m = 0..mmax, by the device routine of the class kernels (mjk_boys).
    T: 1-D float64; returns (n, mmax + 1) float64 on the device."""
    import torch
    T = torch.as_tensor(T, dtype=torch.float64, device=f"cuda:{device}").contiguous().reshape(-1)
    F = torch.empty((T.numel(), int(mmax) + 1), dtype=torch.float64, device=T.device)
    _check(lib().mjk_boys(context(device), int(mmax), ctypes.c_void_p(T.data_ptr()), T.numel(),
                          ctypes.c_void_p(F.data_ptr()), _stream(torch, device)))
    return F


class Plan:
    """A bound plan: tables for one basis/geometry in a torch-owned workspace."""

    def __init__(self, basis: dict, tau: float = 0.0, flags: int = 0, device: int = 0, fp32_tau: float = 0.0,
                 grad: bool = False):
        import torch
        if grad:
            flags |= FLAG_GRAD
        self.torch = torch
        self.device = device
        self.basis = basis
        self.tau = float(tau)
        self._hb = _HostBasis(basis)
        ctx = context(device)
        opts = JKOpts(float(tau), float(fp32_tau), int(flags))
        p = ctypes.c_void_p()
        nbytes = ctypes.c_size_t(0)
        _check(lib().mjk_plan_create(ctx, ctypes.byref(self._hb.s), ctypes.byref(opts), ctypes.byref(p),
                                     ctypes.byref(nbytes)))
        self._p = p
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=f"cuda:{device}")
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        _check(lib().mjk_plan_bind(p, ctypes.c_void_p(aligned), ctypes.c_size_t(int(nbytes.value)),
                                   _stream(torch, device)))
        st = PlanStats()
        _check(lib().mjk_plan_stats_get(p, ctypes.byref(st)))
        self.stats = st.as_dict()
        self.nbf = int(st.nbf)

    def __del__(self):
        p = getattr(self, "_p", None)
        if p is not None and p.value and _lib is not None:
            _lib.mjk_plan_destroy(p)
            self._p = None

    def build_jk(self, D, J=None, K=None):
        """J, K (torch float64 on the plan's device) for symmetric density D."""
        torch = self.torch
        D = torch.as_tensor(D, dtype=torch.float64, device=f"cuda:{self.device}").contiguous()
        n = self.nbf
        if D.shape != (n, n):
            raise MjkError(-1, f"D has shape {tuple(D.shape)}, expected ({n}, {n})")
        if J is None:
            J = torch.empty((n, n), dtype=torch.float64, device=D.device)
        if K is None:
            K = torch.empty((n, n), dtype=torch.float64, device=D.device)
        _check(lib().mjk_build_jk(self._p, ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(J.data_ptr()),
                                  ctypes.c_void_p(K.data_ptr()), _stream(torch, self.device)))
        return J, K

    def build_jk_static(self, D, J, K):
        """J, K into the caller's J, K through mjk_build_jk_static (the library's
        static scratch; the call allocates nothing).  D, J, K: contiguous
        float64 (nbf, nbf) tensors on the plan's device."""
        _check(lib().mjk_build_jk_static(self._p, self._dev_matrix(D, "D"), self._dev_matrix(J, "J"),
                                         self._dev_matrix(K, "K"), _stream(self.torch, self.device)))
        return J, K

    def _dev_matrix(self, M, name):
        torch = self.torch
        n = self.nbf
        if not (torch.is_tensor(M) and M.dtype == torch.float64 and M.is_contiguous()
                and M.device == torch.device(f"cuda:{self.device}") and M.shape == (n, n)):
            raise MjkError(-1, f"{name} must be a contiguous float64 ({n}, {n}) tensor on cuda:{self.device}")
        return ctypes.c_void_p(M.data_ptr())

    def e2(self, D, J, K, out=None):
        """E2 = 1/2 Tr(DJ) - 1/4 Tr(DK) as a 0-d device tensor (mjk_e2)."""
        torch = self.torch
        if out is None:
            out = torch.empty((), dtype=torch.float64, device=f"cuda:{self.device}")
        _check(lib().mjk_e2(self._p, self._dev_matrix(D, "D"), self._dev_matrix(J, "J"), self._dev_matrix(K, "K"),
                            ctypes.c_void_p(out.data_ptr()), _stream(torch, self.device)))
        return out

    def grad_e2(self, D, out=None):
        """dE2/dR at fixed D, (natom, 3) float64 on the plan's device (mjk_grad_e2)."""
        torch = self.torch
        natom = self._hb.xyz.shape[0]
        if out is None:
            out = torch.empty((natom, 3), dtype=torch.float64, device=f"cuda:{self.device}")
        _check(lib().mjk_grad_e2(self._p, self._dev_matrix(D, "D"), ctypes.c_void_p(out.data_ptr()),
                                 _stream(torch, self.device)))
        return out

    def e2_backward(self, D, J=None, K=None, gout=None, want_D=True, want_R=True):
        """(gD, gR) = gout * (dE2/dD, dE2/dR) from the library (mjk_e2_backward);
        gout: 0-d float64 tensor on the plan's device or None (= 1)."""
        torch = self.torch
        dev = f"cuda:{self.device}"
        gD = torch.empty((self.nbf, self.nbf), dtype=torch.float64, device=dev) if want_D else None
        gR = torch.empty((self._hb.xyz.shape[0], 3), dtype=torch.float64, device=dev) if want_R else None
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p()  # noqa: E731
        if gout is not None and not (torch.is_tensor(gout) and gout.dtype == torch.float64 and gout.numel() == 1
                                     and gout.device == torch.device(dev)):
            raise MjkError(-1, f"gout must be one float64 value on {dev}")
        _check(lib().mjk_e2_backward(self._p, self._dev_matrix(D, "D") if want_R else ctypes.c_void_p(),
                                     self._dev_matrix(J, "J") if want_D else ctypes.c_void_p(),
                                     self._dev_matrix(K, "K") if want_D else ctypes.c_void_p(),
                                     ptr(gout), ptr(gD), ptr(gR), _stream(torch, self.device)))
        return gD, gR

    def eri_class(self, quartets):
        """Contracted ERI blocks for shell quartets (nq x 4), as a list of (na,nb,nc,nd) tensors."""
        torch = self.torch
        q = np.ascontiguousarray(np.asarray(quartets, dtype=np.int32).reshape(-1, 4))
        nc = self._hb.ncart
        sizes = [int(nc[a] * nc[b] * nc[c] * nc[d]) for a, b, c, d in q] if len(q) else []
        total = int(sum(sizes))
        out = torch.empty(max(total, 1), dtype=torch.float64, device=f"cuda:{self.device}")
        _check(lib().mjk_eri_class(self._p, q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(q),
                                   ctypes.c_void_p(out.data_ptr()), total, _stream(torch, self.device)))
        res, o = [], 0
        for (a, b, c, d), s in zip(q, sizes):
            res.append(out[o:o + s].view(int(nc[a]), int(nc[b]), int(nc[c]), int(nc[d])))
            o += s
        return res

    def set_tiles(self, qpl):
        """Quartets per lane (mjk_plan_set_tiles): num_classes() ints, or
        num_classes() * mjk_num_kbuckets() (per class and bra K-bucket)."""
        arr = (ctypes.c_int32 * len(qpl))(*[int(v) for v in qpl])
        _check(lib().mjk_plan_set_tiles(self._p, arr, len(qpl)))

    def set_timing(self, enable: bool = True):
        _check(lib().mjk_plan_set_timing(self._p, int(bool(enable))))

    def timings(self):
        """Per-class kernel times of the last build_jk (call after the stream completed)."""
        cap = 256
        arr = (ClassTiming * cap)()
        n = ctypes.c_int32(0)
        _check(lib().mjk_plan_timings(self._p, arr, cap, ctypes.byref(n)))
        return [arr[i].as_dict() for i in range(min(n.value, cap))]

    def set_density_screen(self, dD, tau: float | None = None):
        """Density-weighted screening by the density change dD (contiguous
        float64 (nbf, nbf) on the plan's device) at threshold tau (default:
        the plan's Schwarz threshold), or dD = None to restore the plain work
        lists (mjk_plan_set_density_screen); `stats` follows the new lists."""
        ptr = self._dev_matrix(dD, "dD") if dD is not None else ctypes.c_void_p()
        t = self.tau if tau is None else float(tau)
        _check(lib().mjk_plan_set_density_screen(self._p, ptr, ctypes.c_double(t), _stream(self.torch, self.device)))
        st = PlanStats()
        _check(lib().mjk_plan_stats_get(self._p, ctypes.byref(st)))
        self.stats = st.as_dict()

    def kept_quartets(self) -> int:
        """Unique shell quartets the current work lists run."""
        st = PlanStats()
        _check(lib().mjk_plan_stats_get(self._p, ctypes.byref(st)))
        return int(st.nquartet_kept)

    def one_electron(self, Z):
        """(S, T, V, E_nuc): overlap, kinetic-energy and nuclear-attraction
        matrices (nbf, nbf) and the nuclear repulsion (0-d), float64 on the
        plan's device (mjk_one_electron); Z: one charge per atom."""
        torch = self.torch
        dev = f"cuda:{self.device}"
        natom = self._hb.xyz.shape[0]
        Z = torch.as_tensor(Z, dtype=torch.float64).reshape(-1).to(dev).contiguous()
        if Z.numel() != natom:
            raise MjkError(-1, f"Z has {Z.numel()} values, expected {natom}")
        if not bool(torch.isfinite(Z).all()):
            raise MjkError(-1, "Z must be finite")
        n = self.nbf
        S, T, V = (torch.empty((n, n), dtype=torch.float64, device=dev) for _ in range(3))
        enuc = torch.empty((), dtype=torch.float64, device=dev)
        p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
        _check(lib().mjk_one_electron(self._p, p(Z), p(S), p(T), p(V), p(enuc), _stream(torch, self.device)))
        return S, T, V, enuc

    def schwarz(self):
        ns = len(self._hb.l)
        Q = np.zeros((ns, ns))
        _check(lib().mjk_schwarz(self._p, Q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return Q


def num_classes() -> int:
    return int(lib().mjk_num_classes())


def class_names():
    """Quartet class names ("ssss", "psss", ...) in the library's class order."""
    out = []
    l4 = (ctypes.c_int32 * 4)()
    for q in range(num_classes()):
        _check(lib().mjk_class_l(q, l4))
        out.append("".join("spdfg"[l4[i]] for i in range(4)))
    return out


class Batch:
    """Many molecules in one launch per class (mjk_batch_*).  D, J, K of
    molecule m are views into one packed device buffer (offsets())."""

    def __init__(self, bases, tau: float = 0.0, device: int = 0, fp32_tau: float = 0.0, flags: int = 0):
        import torch
        self.torch = torch
        self.device = device
        self._hbs = [_HostBasis(b) for b in bases]
        n = len(self._hbs)
        arr = (Basis * n)(*[h.s for h in self._hbs])
        opts = JKOpts(float(tau), float(fp32_tau), int(flags))
        p = ctypes.c_void_p()
        nbytes = ctypes.c_size_t(0)
        _check(lib().mjk_batch_create(context(device), n, arr, ctypes.byref(opts), ctypes.byref(p),
                                      ctypes.byref(nbytes)))
        self._b = p
        self.nmol = n
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=f"cuda:{device}")
        aligned = (self.workspace.data_ptr() + 255) & ~255
        _check(lib().mjk_batch_bind(p, ctypes.c_void_p(aligned), ctypes.c_size_t(int(nbytes.value)),
                                    _stream(torch, device)))
        off = (ctypes.c_int64 * (n + 1))()
        _check(lib().mjk_batch_offsets(p, off))
        self.mat_off = [int(off[i]) for i in range(n + 1)]
        self.nbf = [int(h.ncart.sum()) for h in self._hbs]
        st = PlanStats()
        nq = (ctypes.c_int64 * n)()
        _check(lib().mjk_batch_stats(p, ctypes.byref(st), nq))
        self.stats = st.as_dict()
        self.nq_per_mol = [int(nq[i]) for i in range(n)]

    def __del__(self):
        b = getattr(self, "_b", None)
        if b is not None and b.value and _lib is not None:
            _lib.mjk_batch_destroy(b)
            self._b = None

    def pack(self, Ds):
        """One packed float64 device buffer from per-molecule matrices."""
        torch = self.torch
        buf = torch.empty(self.mat_off[-1], dtype=torch.float64, device=f"cuda:{self.device}")
        for m, D in enumerate(Ds):
            buf[self.mat_off[m]:self.mat_off[m + 1]] = torch.as_tensor(
                D, dtype=torch.float64, device=buf.device).reshape(-1)
        return buf

    def unpack(self, buf):
        return [buf[self.mat_off[m]:self.mat_off[m + 1]].view(self.nbf[m], self.nbf[m]) for m in range(self.nmol)]

    def _buf(self, x, name):
        torch = self.torch
        if not (torch.is_tensor(x) and x.dtype == torch.float64 and x.is_contiguous() and x.numel() == self.mat_off[-1]
                and x.device == torch.device(f"cuda:{self.device}")):
            raise MjkError(-1, f"{name} must be a packed contiguous float64 tensor of {self.mat_off[-1]} elements")
        return ctypes.c_void_p(x.data_ptr())

    def build_jk(self, D, J=None, K=None):
        """Packed J, K for the packed density D (mjk_batch_build_jk)."""
        torch = self.torch
        if J is None:
            J = torch.empty_like(D)
        if K is None:
            K = torch.empty_like(D)
        _check(lib().mjk_batch_build_jk(self._b, self._buf(D, "D"), self._buf(J, "J"), self._buf(K, "K"),
                                        _stream(torch, self.device)))
        return J, K

    def set_tiles(self, qpl):
        arr = (ctypes.c_int32 * len(qpl))(*[int(v) for v in qpl])
        _check(lib().mjk_batch_set_tiles(self._b, arr, len(qpl)))

    def autotune(self, D, reps: int = 2, per_bucket: bool = True, cache: str | None = None,
                 key: str | None = None, min_share: float = 0.01, log=None):
        """Algorithm 2 on this batch (mjk_batch_autotune); returns the chosen
        quartets-per-lane table (left active): one value per (class, bra
        K-bucket) with per_bucket, else per class.

        The classes are tuned one call at a time, costliest first (`log`, if
        given, receives a line per class); classes taking less than
        `min_share` of one build keep one quartet per lane.  cache: path of a
        JSON file of tables from earlier runs, keyed by the device
        architecture, the build's class count, the table layout and `key`
        (the caller's name for the workload).  A table found there is set
        without tuning; a new one is added to the file."""
        torch = self.torch
        nkb = lib().mjk_num_kbuckets() if per_bucket else 1
        n = num_classes() * nkb
        ckey = None
        if cache is not None:
            arch = torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
            ckey = f"{arch}/classes{num_classes()}/{'class-kbucket' if per_bucket else 'class'}/{key or 'default'}"
            table = _cache_read(cache).get(ckey)
            if table is not None and len(table) == n:
                self.set_tiles(table)
                return list(table)
        J = torch.empty_like(D)
        K = torch.empty_like(D)
        table = [1] * n
        self.set_tiles(table)
        self.set_timing(True)
        self.build_jk(D, J, K)
        torch.cuda.synchronize(self.device)
        ms = {t["cls"]: t["ms"] for t in self.timings()}
        self.set_timing(False)
        names = class_names()
        total = sum(ms.values())
        for q in sorted(range(num_classes()), key=lambda q: -ms.get(names[q], 0.0)):
            if ms.get(names[q], 0.0) < min_share * total:
                continue
            io = list(table)
            for k in range(nkb):
                io[q * nkb + k] = 0
            arr = (ctypes.c_int32 * n)(*io)
            _check(lib().mjk_batch_autotune(self._b, self._buf(D, "D"), self._buf(J, "J"), self._buf(K, "K"),
                                            int(reps), arr, n, _stream(torch, self.device)))
            table = [int(arr[i]) for i in range(n)]
            if log is not None:
                log(f"autotune {names[q]} ({ms[names[q]]:.1f} ms at 1 quartet per lane): "
                    f"{table[q * nkb:(q + 1) * nkb]}")
        if ckey is not None:
            entries = _cache_read(cache)
            entries[ckey] = table
            tmp = cache + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(entries, fh, indent=1)
            os.replace(tmp, cache)
        return table

    def set_stamps(self, enable: bool = True):
        _check(lib().mjk_batch_set_stamps(self._b, int(bool(enable))))

    def mol_times(self):
        """(start_ms, end_ms) per molecule of the last build, from the earliest start."""
        ms = (ctypes.c_double * (2 * self.nmol))()
        _check(lib().mjk_batch_mol_times(self._b, ms))
        return [(ms[2 * m], ms[2 * m + 1]) for m in range(self.nmol)]

    def set_timing(self, enable: bool = True):
        _check(lib().mjk_batch_set_timing(self._b, int(bool(enable))))

    def timings(self):
        cap = 256
        arr = (ClassTiming * cap)()
        n = ctypes.c_int32(0)
        _check(lib().mjk_batch_timings(self._b, arr, cap, ctypes.byref(n)))
        return [arr[i].as_dict() for i in range(min(n.value, cap))]


_E2 = None


def _e2_function():
    """torch.autograd.Function E2(coords, D, basis, tau=0, device=0).

    forward: plan for the basis at `coords` (natom x 3, bohr), J and K
    (mjk_build_jk), E2 = 1/2 Tr(DJ) - 1/4 Tr(DK) (mjk_e2).
    backward: mjk_e2_backward, which returns the upstream gradient times
    dE2/dcoords (at fixed D) and times dE2/dD = J - K/2 (the derivative with
    respect to a symmetric D's entries, taken as independent).  The results
    are handed back on the inputs' devices and dtypes."""
    global _E2
    if _E2 is not None:
        return _E2
    import torch

    class E2(torch.autograd.Function):
        @staticmethod
        def forward(ctx, coords, D, basis, tau=0.0, device=0):
            b = dict(basis)
            b["xyz"] = coords.detach().to("cpu", torch.float64).numpy().reshape(-1, 3)
            plan = Plan(b, tau=tau, device=device, grad=True)
            Dd = D.detach().to(f"cuda:{device}", torch.float64).contiguous()
            J, K = plan.build_jk(Dd)
            e = plan.e2(Dd, J, K)
            ctx.plan = plan
            ctx.coords_meta = (coords.shape, coords.dtype, coords.device)
            ctx.D_meta = (D.dtype, D.device)
            ctx.save_for_backward(Dd, J, K)
            return e.to(D.device) if D.device != e.device else e

        @staticmethod
        def backward(ctx, g):
            Dd, J, K = ctx.saved_tensors
            shape, dtype, dev = ctx.coords_meta
            want_R, want_D = bool(ctx.needs_input_grad[0]), bool(ctx.needs_input_grad[1])
            gc = gD = None
            if want_R or want_D:
                gout = g.detach().to(Dd.device, torch.float64).reshape(()).contiguous()
                gD, gR = ctx.plan.e2_backward(Dd, J, K, gout, want_D=want_D, want_R=want_R)
                if want_R:
                    gc = gR.reshape(shape).to(dev, dtype)
                if want_D:
                    gD = gD.to(ctx.D_meta[1], ctx.D_meta[0])
            return gc, gD, None, None, None

    _E2 = E2
    return E2


def __getattr__(name):
    if name == "E2":
        return _e2_function()
    raise AttributeError(name)


def build_jk(basis: dict, D, tau: float = 0.0, device: int = 0):
    """One-shot J, K for `basis` and density `D` (plans and binds each call)."""
    plan = Plan(basis, tau=tau, device=device)
    return plan.build_jk(D)


def eri_class(basis: dict, quartets, device: int = 0):
    return Plan(basis, device=device).eri_class(quartets)
