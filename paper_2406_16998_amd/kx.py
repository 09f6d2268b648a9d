"""Thin ctypes binding of libkx (include/kx.h): argument marshalling only.

Every numerical step runs inside the HIP library.  PyTorch supplies device
memory and the stream.  If libkx.so is missing this module raises on first
use; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkx.so")

KX_OK = 0
STATUS = {
    0: "KX_OK", 1: "KX_ERR_INVALID_ARG", 2: "KX_ERR_UNSUPPORTED", 3: "KX_ERR_SINGULAR",
    4: "KX_ERR_OUT_OF_MEMORY", 5: "KX_ERR_DEVICE", 6: "KX_ERR_STATE", 7: "KX_ERR_NUMERIC",
}
BC = {"dirichlet": 0, "periodic": 1}
KERNEL = {"coulomb": 0, "erfc": 1}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x3": 3, "mixed": 4}
DTYPE = {"f64": 0, "f32": 1}

# every symbol include/kx.h declares
EXPORTS = (
    "kx_setup_laplacian", "kx_apply_fL", "kx_apply_exchange", "kx_exchange_energy",
    "kx_pair_energies", "kx_get_eigensystem", "kx_destroy", "kx_status_string",
    "kx_fd_weights", "kx_laplacian_1d", "kx_pair_schedule", "kx_profile", "kx_profile_read",
    "kx_batch_apply_exchange", "kx_autotune", "kx_get_plan", "kx_ace_build", "kx_ace_apply",
    "kx_profile_phases", "kx_reserve", "kx_apply_exchange_noalloc", "kx_apply_fL_multipole",
    "kx_reserve_bloch", "kx_apply_fL_bloch", "kx_apply_exchange_bloch", "kx_set_cell",
    "kx_set_checks", "kx_apply_exchange_multipole", "kx_set_zero_mode",
    "kx_ace_build_complex", "kx_ace_apply_complex",
)
PHASE = {"forward": 0, "pencil": 1, "inverse": 2, "energy": 3, "accum": 4}


class KxError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}")


_lib = None


def lib():
    """Load libkx.so (after torch, so one HIP runtime serves both)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
        try:
            import torch  # noqa: F401  (load torch's HIP runtime first)
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        c_int, c_double, vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        ip, dp = ctypes.POINTER(c_int), ctypes.POINTER(c_double)
        sig = {
            "kx_setup_laplacian": [ip, dp, c_int, ip, vp, ctypes.POINTER(vp)],
            "kx_apply_fL": [vp, c_int, c_double, c_int, c_int, vp, vp, c_int],
            "kx_apply_exchange": [vp, c_int, c_double, c_int, c_int, vp, dp, vp, c_int],
            "kx_apply_exchange_noalloc": [vp, c_int, c_double, c_int, c_int, vp, dp, vp, c_int],
            "kx_reserve": [vp, c_int, c_int, c_int],
            "kx_apply_fL_multipole": [vp, c_int, c_int, vp, vp, c_int, c_int, dp],
            "kx_reserve_bloch": [vp, c_int, c_int],
            "kx_set_cell": [vp, dp],
            "kx_set_checks": [vp, c_int],
            "kx_set_zero_mode": [vp, c_int, c_double],
            "kx_ace_build_complex": [vp, c_int, vp, vp, vp],
            "kx_ace_apply_complex": [vp, c_int, vp, c_int, vp, vp],
            "kx_apply_exchange_multipole": [vp, c_int, c_int, vp, dp, vp, c_int, c_int, dp],
            "kx_apply_fL_bloch": [vp, c_int, c_double, c_int, dp, vp, vp, c_int],
            "kx_apply_exchange_bloch": [vp, c_int, c_double, c_int, c_int, dp, dp, dp, vp, vp,
                                        c_int],
            "kx_exchange_energy": [vp, dp],
            "kx_pair_energies": [vp, c_int, ip, dp],
            "kx_get_eigensystem": [vp, c_int, dp, dp],
            "kx_destroy": [vp],
            "kx_status_string": [c_int],
            "kx_fd_weights": [c_int, dp],
            "kx_laplacian_1d": [c_int, c_double, c_int, c_int, dp],
            "kx_pair_schedule": [c_int, c_int, ip, ip, ip, ip],
            "kx_autotune": [vp, c_int, c_int, c_int, c_int, ctypes.c_char_p],
            "kx_get_plan": [vp, c_int, ip, ip, ip],
            "kx_batch_apply_exchange": [c_int, ctypes.POINTER(vp), ip, dp, ip, c_int,
                                        ctypes.POINTER(vp), ctypes.POINTER(dp),
                                        ctypes.POINTER(vp), c_int, dp],
            "kx_profile": [vp, c_int],
            "kx_profile_phases": [vp, c_int],
            "kx_ace_build": [vp, c_int, c_int, vp, vp, vp],
            "kx_ace_apply": [vp, c_int, c_int, vp, c_int, vp, vp],
            "kx_profile_read": [vp, c_int, dp, ctypes.POINTER(ctypes.c_longlong)],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name == "kx_status_string" else c_int
        _lib = L
    return _lib


def _check(st, where):
    if st != KX_OK:
        raise KxError(st, where)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _span(t):
    a = t.data_ptr()
    return a, a + t.numel() * t.element_size()


def check_fields(t, shape3, device, name, batch_dims=1):
    """Raise ValueError unless t is a contiguous float32/float64 tensor on the
    handle's device with shape (batch, n3, n2, n1).  Returns the library's
    storage code.  Runs before any library call, so that a host tensor, a
    wrong shape or dtype never reaches a kernel as a raw pointer."""
    import torch
    if not isinstance(getattr(t, "dtype", None), torch.dtype):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a device tensor, got one on {t.device}")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name}: on cuda:{t.device.index}, the handle was set up on cuda:{device}")
    if t.dtype not in (torch.float32, torch.float64):
        raise ValueError(f"{name}: dtype must be float32 or float64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.dim() != 3 + batch_dims or tuple(t.shape[batch_dims:]) != tuple(shape3):
        raise ValueError(f"{name}: shape {tuple(t.shape)} is not (batch,) + {tuple(shape3)}")
    return DTYPE["f64" if t.dtype == torch.float64 else "f32"]


def check_complex_fields(t, shape3, device, name, batch_dims=1):
    """As check_fields, for complex128 tensors of shape batch + (n3, n2, n1)
    (interleaved real and imaginary parts)."""
    import torch
    if not isinstance(getattr(t, "dtype", None), torch.dtype):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a device tensor, got one on {t.device}")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name}: on cuda:{t.device.index}, the handle was set up on cuda:{device}")
    if t.dtype != torch.complex128:
        raise ValueError(f"{name}: dtype must be complex128, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.dim() != 3 + batch_dims or tuple(t.shape[batch_dims:]) != tuple(shape3):
        raise ValueError(f"{name}: shape {tuple(t.shape)} is not batch + {tuple(shape3)}")


def check_out(out, src, name="out"):
    """out must match src in dtype, shape and device and must not overlap it."""
    if out.dtype != src.dtype or tuple(out.shape) != tuple(src.shape) or out.device != src.device:
        raise ValueError(f"{name}: must match the input's dtype, shape and device "
                         f"({src.dtype}, {tuple(src.shape)}, {src.device}); got "
                         f"({out.dtype}, {tuple(out.shape)}, {out.device})")
    if not out.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    a0, a1 = _span(src)
    b0, b1 = _span(out)
    if src.numel() > 0 and a0 < b1 and b0 < a1:
        raise ValueError(f"{name}: overlaps the input")


def check_occ(occ, norb):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(occ, dtype=np.float64).reshape(-1))
    if a.shape[0] != norb:
        raise ValueError(f"occ: {a.shape[0]} values for {norb} orbitals")
    if not np.all(np.isfinite(a)):
        raise ValueError("occ: values must be finite")
    return a


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


# ---------------------------------------------------------------- host-only
def fd_weights(order):
    import numpy as np
    w = np.zeros(order // 2 + 1)
    _check(lib().kx_fd_weights(order, _dptr(w)), "kx_fd_weights")
    return w


def laplacian_1d(n, h, order, bc):
    import numpy as np
    L = np.zeros((n, n))
    _check(lib().kx_laplacian_1d(n, float(h), order, BC.get(bc, bc), _dptr(L)), "kx_laplacian_1d")
    return L


def pair_schedule(norb, max_batch=0):
    import numpy as np
    npairs, nb = ctypes.c_int(), ctypes.c_int()
    _check(lib().kx_pair_schedule(norb, max_batch, ctypes.byref(npairs), ctypes.byref(nb), None, None),
           "kx_pair_schedule")
    pairs = np.zeros((max(npairs.value, 1), 2), dtype=np.int32)
    offs = np.zeros(nb.value + 1, dtype=np.int32)
    _check(lib().kx_pair_schedule(norb, max_batch, ctypes.byref(npairs), ctypes.byref(nb),
                                  _iptr(pairs), _iptr(offs)), "kx_pair_schedule")
    return pairs[:npairs.value], offs


def batch_apply_exchange(grids, psis, occs, kernels, omegas, prec="fp64", outs=None):
    """Exchange of several systems through kx_batch_apply_exchange (one
    recorded graph, replayed while nothing changes).  Returns (vx list, E_x
    list)."""
    import numpy as np
    import torch
    n = len(grids)
    if not (len(psis) == len(occs) == len(kernels) == len(omegas) == n):
        raise ValueError("one psi, occ, kernel and omega per grid")
    if outs is None:
        outs = [torch.empty_like(p) for p in psis]
    if len(outs) != n:
        raise ValueError("one output per grid")
    for k, (g, p, o) in enumerate(zip(grids, psis, outs)):
        check_fields(p, g.shape3, g.device, f"psis[{k}]")
        check_out(o, p, f"outs[{k}]")
    if len({p.dtype for p in psis}) != 1:
        raise ValueError("psis: one dtype for every system")
    dtype = DTYPE["f64" if psis[0].dtype == torch.float64 else "f32"]
    occ_arrays = [check_occ(o, int(p.shape[0])) for o, p in zip(occs, psis)]
    norbs = (ctypes.c_int * n)(*[int(p.shape[0]) for p in psis])
    ks = (ctypes.c_int * n)(*[KERNEL[k] for k in kernels])
    oms = (ctypes.c_double * n)(*[float(w) for w in omegas])
    hs = (ctypes.c_void_p * n)(*[g._h.value for g in grids])
    ps = (ctypes.c_void_p * n)(*[p.data_ptr() for p in psis])
    vs = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    occ_ptrs = (ctypes.POINTER(ctypes.c_double) * n)(*[_dptr(a) for a in occ_arrays])
    ex = (ctypes.c_double * n)()
    for g in grids:
        g.stream.synchronize()
    _check(lib().kx_batch_apply_exchange(n, hs, ks, oms, norbs, dtype, ps, occ_ptrs, vs, PREC[prec],
                                         ex), "kx_batch_apply_exchange")
    return outs, list(ex)


# ---------------------------------------------------------------- device
class Grid:
    """One kx_grid handle (Laplacian eigensystems, f table, workspace)."""

    def __init__(self, n, h, order, bc, stream=None):
        import numpy as np
        import torch
        self.n = tuple(int(v) for v in n)
        self.h = tuple(float(v) for v in h)
        self.order = int(order)
        self.bc = tuple(bc)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        n_c = (ctypes.c_int * 3)(*self.n)
        h_c = (ctypes.c_double * 3)(*self.h)
        bc_c = (ctypes.c_int * 3)(*[BC.get(b, b) for b in self.bc])
        handle = ctypes.c_void_p()
        st = lib().kx_setup_laplacian(n_c, h_c, self.order, bc_c, ctypes.c_void_p(stream.cuda_stream),
                                      ctypes.byref(handle))
        _check(st, "kx_setup_laplacian")
        self._h = handle
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.shape3 = (self.n[2], self.n[1], self.n[0])
        self.device = torch.cuda.current_device()
        self._np = np

    def close(self):
        if getattr(self, "_h", None):
            lib().kx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def reserve(self, norb, prec="fp64", dtype="f64"):
        """kx_reserve: workspace for later calls on up to norb orbitals (0:
        batches of fields) in precision prec on storage dtype."""
        _check(lib().kx_reserve(self._h, int(norb), PREC[prec], DTYPE[dtype]), "kx_reserve")

    def apply_fL(self, rho, kernel, omega=0.0, prec="fp64", out=None, reserve=True):
        """phi = f(-L) rho; rho is a (batch, n3, n2, n1) device tensor.  With
        reserve=False the workspace must already be reserved (for work
        recorded into a graph)."""
        import torch
        dt = check_fields(rho, self.shape3, self.device, "rho")
        if out is None:
            out = torch.empty_like(rho)
        check_out(out, rho)
        if reserve:
            self.reserve(0, prec, "f64" if dt == DTYPE["f64"] else "f32")
        st = lib().kx_apply_fL(self._h, KERNEL[kernel], float(omega), rho.shape[0], dt, _ptr(rho),
                               _ptr(out), PREC[prec])
        _check(st, "kx_apply_fL")
        return out

    def apply_fL_multipole(self, rho, centre=None, lmax=6, prec="fp64", out=None, reserve=True):
        """phi = (-L_D)^{-1} (4 pi rho + c): the unscreened potential of the
        densities rho (batch, n3, n2, n1) with Dirichlet values from the
        multipole expansion about centre (default: the grid's centre, node i
        of axis k at i h_k)."""
        import numpy as np
        import torch
        dt = check_fields(rho, self.shape3, self.device, "rho")
        if out is None:
            out = torch.empty_like(rho)
        check_out(out, rho)
        if centre is None:
            centre = [(self.n[k] - 1) * self.h[k] / 2 for k in range(3)]
        c = np.ascontiguousarray(np.asarray(centre, dtype=np.float64).reshape(3))
        if reserve:
            self.reserve(0, prec, "f64" if dt == DTYPE["f64"] else "f32")
        st = lib().kx_apply_fL_multipole(self._h, rho.shape[0], dt, _ptr(rho), _ptr(out), PREC[prec],
                                         int(lmax), _dptr(c))
        _check(st, "kx_apply_fL_multipole")
        return out

    def ace_build_complex(self, psi, w, out=None):
        """Compressed exchange of one k-point: psi and W = (Vx psi) complex128
        of shape (norb, n3, n2, n1); returns xi, 2 norb complex fields (the
        real form of the operator's vectors)."""
        import torch
        check_complex_fields(psi, self.shape3, self.device, "psi")
        check_complex_fields(w, self.shape3, self.device, "w")
        if w.shape != psi.shape:
            raise ValueError("w: must match psi's shape")
        norb = psi.shape[0]
        if out is None:
            out = torch.empty((2 * norb,) + tuple(psi.shape[1:]), dtype=psi.dtype, device=psi.device)
        check_complex_fields(out, self.shape3, self.device, "out")
        if out.shape[0] != 2 * norb:
            raise ValueError("out: must hold 2 norb fields")
        for src, name in ((psi, "psi"), (w, "w")):
            a0, a1 = _span(src)
            b0, b1 = _span(out)
            if a0 < b1 and b0 < a1:
                raise ValueError(f"out: overlaps {name}")
        _check(lib().kx_ace_build_complex(self._h, norb, _ptr(psi), _ptr(w), _ptr(out)),
               "kx_ace_build_complex")
        return out

    def ace_apply_complex(self, xi, phi, out=None):
        """V_ACE phi for complex128 phi (nvec, n3, n2, n1), xi from
        ace_build_complex."""
        import torch
        check_complex_fields(xi, self.shape3, self.device, "xi")
        check_complex_fields(phi, self.shape3, self.device, "phi")
        if xi.shape[0] % 2:
            raise ValueError("xi: must hold 2 norb fields")
        if out is None:
            out = torch.empty_like(phi)
        check_out(out, phi)
        a0, a1 = _span(xi)
        b0, b1 = _span(out)
        if a0 < b1 and b0 < a1:
            raise ValueError("out: overlaps xi")
        _check(lib().kx_ace_apply_complex(self._h, xi.shape[0] // 2, _ptr(xi), phi.shape[0],
                                          _ptr(phi), _ptr(out)), "kx_ace_apply_complex")
        return out

    def set_zero_mode(self, value=None):
        """kx_set_zero_mode: f at the zero mode of the unscreened kernel (None:
        off, the singular case is refused)."""
        _check(lib().kx_set_zero_mode(self._h, 0 if value is None else 1,
                                      0.0 if value is None else float(value)), "kx_set_zero_mode")

    def set_checks(self, finite=True):
        """kx_set_checks: KX_CHECK_FINITE on or off."""
        _check(lib().kx_set_checks(self._h, 1 if finite else 0), "kx_set_checks")

    def set_cell(self, lattice=None):
        """kx_set_cell: lattice directions as rows (3 x 3), None for the
        orthogonal cell."""
        import numpy as np
        if lattice is None:
            _check(lib().kx_set_cell(self._h, None), "kx_set_cell")
            return
        a = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(9))
        _check(lib().kx_set_cell(self._h, _dptr(a)), "kx_set_cell")

    def reserve_bloch(self, nk=0, norb=0):
        """kx_reserve_bloch: buffers of the Bloch calls (nk = 0: fields only)."""
        _check(lib().kx_reserve_bloch(self._h, int(nk), int(norb)), "kx_reserve_bloch")

    def apply_fL_bloch(self, rho, theta, kernel, omega=0.0, prec="fp64", out=None, reserve=True):
        """phi = f(-L(theta)) rho for complex128 rho (batch, n3, n2, n1) with
        the Bloch phases theta (radians per axis, 0 on Dirichlet axes)."""
        import numpy as np
        import torch
        check_complex_fields(rho, self.shape3, self.device, "rho")
        if out is None:
            out = torch.empty_like(rho)
        check_out(out, rho)
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(3))
        if reserve:
            self.reserve_bloch(0, 0)
        st = lib().kx_apply_fL_bloch(self._h, KERNEL[kernel], float(omega), rho.shape[0], _dptr(th),
                                     _ptr(rho), _ptr(out), PREC[prec])
        _check(st, "kx_apply_fL_bloch")
        return out

    def apply_exchange_bloch(self, psi, kpts, wk, occ, kernel, omega=0.0, prec="fp64", out=None,
                             reserve=True):
        """(Vx psi)_nk for complex128 psi (nk, norb, n3, n2, n1), reduced
        k-points kpts (nk, 3), weights wk (nk,) and occupations occ (nk, norb)
        (host sequences) of one spin channel.  E_x: exchange_energy()."""
        import numpy as np
        import torch
        check_complex_fields(psi, self.shape3, self.device, "psi", batch_dims=2)
        nk, norb = psi.shape[0], psi.shape[1]
        k = np.ascontiguousarray(np.asarray(kpts, dtype=np.float64))
        w = np.ascontiguousarray(np.asarray(wk, dtype=np.float64))
        o = np.ascontiguousarray(np.asarray(occ, dtype=np.float64))
        if k.shape != (nk, 3) or w.shape != (nk,) or o.shape != (nk, norb):
            raise ValueError(f"kpts, wk, occ: shapes {k.shape}, {w.shape}, {o.shape} are not "
                             f"({nk}, 3), ({nk},), ({nk}, {norb})")
        if out is None:
            out = torch.empty_like(psi)
        check_out(out, psi)
        if reserve:
            self.reserve_bloch(nk, norb)
        st = lib().kx_apply_exchange_bloch(self._h, KERNEL[kernel], float(omega), nk, norb,
                                           _dptr(k), _dptr(w), _dptr(o), _ptr(psi), _ptr(out),
                                           PREC[prec])
        _check(st, "kx_apply_exchange_bloch")
        return out

    def _exchange_args(self, psi, occ, out):
        import torch
        dt = check_fields(psi, self.shape3, self.device, "psi")
        occ_a = check_occ(occ, psi.shape[0])
        if out is None:
            out = torch.empty_like(psi)
        check_out(out, psi)
        return dt, occ_a, out

    def apply_exchange(self, psi, occ, kernel, omega=0.0, prec="fp64", out=None, reserve=True):
        """(Vx psi) for psi of shape (norb, n3, n2, n1); occ a host sequence.
        With reserve=False the workspace must already be reserved (for work
        recorded into a graph)."""
        dt, occ_a, out = self._exchange_args(psi, occ, out)
        norb = psi.shape[0]
        if reserve:
            self.reserve(norb, prec, "f64" if dt == DTYPE["f64"] else "f32")
        st = lib().kx_apply_exchange(self._h, KERNEL[kernel], float(omega), norb, dt, _ptr(psi),
                                     _dptr(occ_a), _ptr(out), PREC[prec])
        _check(st, "kx_apply_exchange")
        return out

    def apply_exchange_multipole(self, psi, occ, centre=None, lmax=6, prec="fp64", out=None,
                                 reserve=True):
        """The unscreened exchange of an isolated system: every pair solve with
        boundary values from the multipole expansion about centre (default:
        the grid's centre).  E_x: exchange_energy()."""
        import numpy as np
        dt, occ_a, out = self._exchange_args(psi, occ, out)
        if centre is None:
            centre = [(self.n[k] - 1) * self.h[k] / 2 for k in range(3)]
        c = np.ascontiguousarray(np.asarray(centre, dtype=np.float64).reshape(3))
        norb = psi.shape[0]
        if reserve:
            self.reserve(norb, prec, "f64" if dt == DTYPE["f64"] else "f32")
        st = lib().kx_apply_exchange_multipole(self._h, norb, dt, _ptr(psi), _dptr(occ_a), _ptr(out),
                                               PREC[prec], int(lmax), _dptr(c))
        _check(st, "kx_apply_exchange_multipole")
        return out

    def apply_exchange_noalloc(self, psi, occ, kernel, omega=0.0, prec="fp64", out=None):
        """kx_apply_exchange_noalloc: the exchange with every per-call buffer in
        the library's fixed device scratch array (out must be given, or is
        allocated here by torch before the call)."""
        dt, occ_a, out = self._exchange_args(psi, occ, out)
        st = lib().kx_apply_exchange_noalloc(self._h, KERNEL[kernel], float(omega), psi.shape[0], dt,
                                             _ptr(psi), _dptr(occ_a), _ptr(out), PREC[prec])
        _check(st, "kx_apply_exchange_noalloc")
        return out

    def exchange_energy(self):
        v = ctypes.c_double()
        _check(lib().kx_exchange_energy(self._h, ctypes.byref(v)), "kx_exchange_energy")
        return v.value

    def ace_build(self, psi, w, out=None):
        """Compressed exchange vectors xi = L^{-1} W, -(psi, W)_h = L L^T,
        for psi and W = Vx psi of shape (norb, n3, n2, n1)."""
        import torch
        dt = check_fields(psi, self.shape3, self.device, "psi")
        check_fields(w, self.shape3, self.device, "w")
        if w.dtype != psi.dtype or w.shape != psi.shape:
            raise ValueError("w: must match psi's dtype and shape")
        if out is None:
            out = torch.empty_like(w)
        check_out(out, w)
        check_out(out, psi)
        st = lib().kx_ace_build(self._h, psi.shape[0], dt, _ptr(psi), _ptr(w), _ptr(out))
        _check(st, "kx_ace_build")
        return out

    def ace_apply(self, xi, phi, out=None):
        """V_ACE phi = -sum_k xi_k (xi_k, phi)_h for phi of shape (nvec, n3, n2, n1)."""
        import torch
        dt = check_fields(xi, self.shape3, self.device, "xi")
        check_fields(phi, self.shape3, self.device, "phi")
        if phi.dtype != xi.dtype:
            raise ValueError("phi: must match xi's dtype")
        if out is None:
            out = torch.empty_like(phi)
        check_out(out, phi)
        a0, a1 = _span(xi)
        b0, b1 = _span(out)
        if a0 < b1 and b0 < a1:
            raise ValueError("out: overlaps xi")
        st = lib().kx_ace_apply(self._h, xi.shape[0], dt, _ptr(xi), phi.shape[0], _ptr(phi),
                                _ptr(out))
        _check(st, "kx_ace_apply")
        return out

    def pair_energies(self, pairs):
        import numpy as np
        p = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        e = np.zeros(len(p))
        _check(lib().kx_pair_energies(self._h, len(p), _iptr(p), _dptr(e)), "kx_pair_energies")
        return e

    def autotune(self, prec="fp64", dtype="f64", items=0, verify=False, cache_path=None):
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(lib().kx_autotune(self._h, PREC[prec], DTYPE[dtype], int(items), 1 if verify else 0,
                                 path), "kx_autotune")

    def plan(self, prec="fp64"):
        """Launch shapes in use: dicts for the forward, pencil and inverse passes."""
        f, p, v = (ctypes.c_int * 6)(), (ctypes.c_int * 3)(), (ctypes.c_int * 6)()
        _check(lib().kx_get_plan(self._h, PREC[prec], f, p, v), "kx_get_plan")
        keys = ("qsplit", "slabs", "waves", "kc", "vlds", "lds_bytes")
        return (dict(zip(keys, list(f))), {"waves": p[0], "lds_bytes": p[1], "per": p[2]},
                dict(zip(keys, list(v))))

    def profile(self, enable=True):
        _check(lib().kx_profile(self._h, 1 if enable else 0), "kx_profile")

    def profile_phases(self, phases):
        """Time only the launches of the named phases (see profile)."""
        mask = 0
        for ph in phases:
            mask |= 1 << PHASE[ph]
        _check(lib().kx_profile_phases(self._h, mask), "kx_profile_phases")

    def profile_read(self, phase):
        """(total ms, launches) of one phase since profile(True)."""
        ms, cnt = ctypes.c_double(), ctypes.c_longlong()
        _check(lib().kx_profile_read(self._h, PHASE[phase], ctypes.byref(ms), ctypes.byref(cnt)),
               "kx_profile_read")
        return ms.value, cnt.value

    def eigensystem(self, axis):
        import numpy as np
        n = self.n[axis]
        lam = np.zeros(n)
        V = np.zeros((n, n))
        _check(lib().kx_get_eigensystem(self._h, axis, _dptr(lam), _dptr(V)), "kx_get_eigensystem")
        return lam, V
