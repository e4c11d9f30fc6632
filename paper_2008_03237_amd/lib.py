"""ctypes binding of include/dlpno.h.  Argument marshalling only."""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))

FP64, FP32, BF16X2, FP16X2 = 0, 1, 2, 3
_PREC = {"fp64": FP64, "fp32": FP32, "bf16x2": BF16X2, "fp16x2": FP16X2}
FLAG_GENERAL_T = 1     # same-spin amplitude blocks need not be antisymmetric
FLAG_QUADRATIC = 2     # quadratic CCSD term over the hole-hole couplings
FLAG_QUADRATIC_OCC = 4  # quadratic part of the occupied Fock intermediate


class DlpnoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("dlpno status %d: %s" % (status, msg))
        self.status = status


class Pair(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("npno", C.c_int32), ("naux", C.c_int32),
                ("blocks", C.c_uint32), ("n_somo_virt", C.c_int32), ("off_B", C.c_int64), ("off_T", C.c_int64),
                ("off_K", C.c_int64), ("off_eps", C.c_int64)]


class Coupling(C.Structure):
    _fields_ = [("src_pair", C.c_int32), ("k", C.c_int32), ("side", C.c_int32), ("reserved", C.c_int32),
                ("off_S", C.c_int64)]


class Problem(C.Structure):
    _fields_ = [("n_occ", C.c_int32), ("n_pairs", C.c_int32), ("n_couplings", C.c_int64),
                ("is_somo", C.c_void_p), ("pairs", C.c_void_p), ("cpl_rowptr", C.c_void_p), ("cpl", C.c_void_p),
                ("f_a", C.c_void_p), ("f_b", C.c_void_p), ("n_B", C.c_int64), ("n_T", C.c_int64),
                ("n_K", C.c_int64), ("n_eps", C.c_int64), ("n_S", C.c_int64),
                ("n_hh", C.c_int64), ("hh_rowptr", C.c_void_p), ("hh", C.c_void_p),
                ("n_ring", C.c_int64), ("ring_rowptr", C.c_void_p), ("ring", C.c_void_p),
                ("n_ring_ints", C.c_int64)]


class Inputs(C.Structure):
    _fields_ = [("B", C.c_void_p), ("S", C.c_void_p), ("K", C.c_void_p), ("eps_a", C.c_void_p),
                ("eps_b", C.c_void_p), ("ring_ints", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("diis_max", C.c_int32), ("diis_start", C.c_int32),
                ("n_workers", C.c_int32), ("items_per_wave", C.c_int32), ("flags", C.c_int32)]


PAIR_DTYPE = np.dtype([("i", "<i4"), ("j", "<i4"), ("npno", "<i4"), ("naux", "<i4"), ("blocks", "<u4"),
                       ("n_somo_virt", "<i4"), ("off_B", "<i8"), ("off_T", "<i8"), ("off_K", "<i8"),
                       ("off_eps", "<i8")])
CPL_DTYPE = np.dtype([("src_pair", "<i4"), ("k", "<i4"), ("side", "<i4"), ("reserved", "<i4"), ("off_S", "<i8")])
HH_DTYPE = np.dtype([("src_pair", "<i4"), ("k", "<i4"), ("l", "<i4"), ("reserved", "<i4"), ("off_S", "<i8"),
                     ("w", "<f8")])
RING_DTYPE = np.dtype([("src_pair", "<i4"), ("m", "<i4"), ("role", "<i4"), ("reserved", "<i4"), ("off_S", "<i8"),
                       ("off_X", "<i8"), ("off_J", "<i8")])

_LIB = None


def library_path():
    """The in-tree libdlpno.so, or the file named by DLPNO_LIBRARY (another
    build of the same sources, e.g. for side-by-side timing)."""
    return os.environ.get("DLPNO_LIBRARY") or os.path.join(_HERE, "libdlpno.so")


def lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ImportError("libdlpno.so is not built (%s); run __graft_entry__.build()" % path)
    L = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "dlpno_plan_create": [C.POINTER(Problem), C.POINTER(Inputs), C.POINTER(Options), vp, C.POINTER(vp)],
        "dlpno_plan_destroy": [vp],
        "dlpno_residual": [vp, vp, vp, vp],
        "dlpno_residual_noalloc": [vp, vp, vp, vp],
        "dlpno_update": [vp, vp, vp, vp, vp, vp, vp],
        "dlpno_f12_energy": [vp, vp, vp, vp, vp, vp, vp],
        "dlpno_iterate": [vp, i32, vp, vp, vp, vp, vp, vp],
        "dlpno_reset": [vp, vp],
        "dlpno_residual_vjp": [vp, vp, vp, vp, vp, vp],
        "dlpno_solve_mixed": [vp, i32, i32, vp, vp, vp, vp, vp, vp],
        "dlpno_flop_count": [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)],
        "dlpno_ring_flop_count": [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
        "dlpno_diis_state": [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double), vp],
        "dlpno_solve": [vp, i32, C.c_double, C.c_double, vp, vp, vp, vp, vp, C.POINTER(C.c_int32), vp],
        "dlpno_checkpoint_size": [vp, C.POINTER(C.c_size_t)],
        "dlpno_checkpoint_save": [vp, vp, vp, vp],
        "dlpno_checkpoint_load": [vp, vp, vp, vp],
        "dlpno_autotune": [vp, vp, vp, vp],
        "dlpno_autotune_cached": [vp, vp, vp, C.c_char_p, C.POINTER(C.c_int32), vp],
        "dlpno_set_profiling": [vp, i32],
        "dlpno_phase_times": [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), i32],
        "dlpno_pno_plan_create": [vp, i64, i64, i64, i64, i64, C.POINTER(vp)],
        "dlpno_pno_build": [vp, vp, vp, C.c_double, vp, vp, vp, vp, vp, vp],
        "dlpno_pno_plan_destroy": [vp],
        "dlpno_pno_overlap_prepare": [vp, vp, vp, vp, vp, i64],
        "dlpno_pno_overlap": [vp, vp, vp, vp],
    }
    for name, args in sig.items():
        # a library built from older sources lacks newer entry points: only
        # calls of those fail (AttributeError), the others keep working
        f = getattr(L, name, None)
        if f is None:
            continue
        f.argtypes = args
        f.restype = C.c_int
    L.dlpno_history.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), i32]
    L.dlpno_history.restype = i32
    L.dlpno_plan_info.argtypes = [vp]
    L.dlpno_plan_info.restype = C.c_char_p
    L.dlpno_status_string.argtypes = [C.c_int]
    L.dlpno_status_string.restype = C.c_char_p
    L.dlpno_last_error.argtypes = []
    L.dlpno_last_error.restype = C.c_char_p
    _LIB = L
    return L


def _check(st):
    if st != 0:
        L = lib()
        raise DlpnoError(st, "%s: %s" % (L.dlpno_status_string(st).decode(), L.dlpno_last_error().decode()))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A residual plan over device-resident inputs (torch CUDA float64 tensors).

    desc: object with the descriptor arrays (n_occ, is_somo, pi, pj, npno, naux,
    blocks, off_B, off_T, off_K, off_eps, cpl_rowptr, cpl_src, cpl_k, cpl_side,
    cpl_off_S, f_a, f_b, n_B, n_T, n_K, n_S and eps sizes), e.g. a
    workload.Problem.  B, S, K, eps_a, eps_b: device tensors (kept referenced).
    The same-spin blocks of the amplitudes passed to residual/iterate must be
    antisymmetric (as physical amplitudes are) unless general_T is set.
    Optional descriptor fields switch on the further CCSD terms: hh_* (the
    hole-hole ladder; with quadratic=True also its quadratic term) and ring_*
    (the ring/exchange term, with its integral blocks in the device tensor
    ring_ints); quadratic_occ=True adds the quadratic part of the occupied
    Fock intermediate (no further inputs).
    """

    def __init__(self, desc, B, S, K, eps_a, eps_b, precision="fp64", diis_max=8, diis_start=3, n_workers=0,
                 items_per_wave=0, general_T=False, quadratic=False, ring_ints=None, quadratic_occ=False):
        import torch
        L = lib()
        P = len(desc.pi)
        pairs = np.zeros(P, dtype=PAIR_DTYPE)
        pairs["i"], pairs["j"], pairs["npno"], pairs["naux"] = desc.pi, desc.pj, desc.npno, desc.naux
        pairs["blocks"] = desc.blocks
        if getattr(desc, "n_sv", None) is not None:
            pairs["n_somo_virt"] = desc.n_sv
        pairs["off_B"], pairs["off_T"], pairs["off_K"], pairs["off_eps"] = desc.off_B, desc.off_T, desc.off_K, desc.off_eps
        ncpl = len(desc.cpl_src)
        cpl = np.zeros(max(ncpl, 1), dtype=CPL_DTYPE)
        cpl["src_pair"][:ncpl], cpl["k"][:ncpl], cpl["side"][:ncpl] = desc.cpl_src, desc.cpl_k, desc.cpl_side
        cpl["off_S"][:ncpl] = desc.cpl_off_S
        # hole-hole ladder couplings (optional descriptor fields)
        nhh = int(getattr(desc, "n_hh", 0) or 0)
        hh = np.zeros(max(nhh, 1), dtype=HH_DTYPE)
        hh_rowptr = np.zeros(P + 1, dtype=np.int64)
        if nhh > 0:
            hh["src_pair"][:nhh], hh["k"][:nhh], hh["l"][:nhh] = desc.hh_src, desc.hh_k, desc.hh_l
            hh["off_S"][:nhh], hh["w"][:nhh] = desc.hh_off_S, desc.hh_w
            hh_rowptr = np.ascontiguousarray(desc.hh_rowptr, dtype=np.int64)
        # ring/exchange couplings (optional descriptor fields; need ring_ints)
        nring = int(getattr(desc, "n_ring", 0) or 0) if ring_ints is not None else 0
        ring = np.zeros(max(nring, 1), dtype=RING_DTYPE)
        ring_rowptr = np.zeros(P + 1, dtype=np.int64)
        if nring > 0:
            ring["src_pair"][:nring], ring["m"][:nring], ring["role"][:nring] = desc.ring_src, desc.ring_m, desc.ring_role
            ring["off_S"][:nring], ring["off_X"][:nring], ring["off_J"][:nring] = (desc.ring_off_S, desc.ring_off_X,
                                                                                   desc.ring_off_J)
            ring_rowptr = np.ascontiguousarray(desc.ring_rowptr, dtype=np.int64)
        self._host = dict(
            somo=np.ascontiguousarray(desc.is_somo, dtype=np.uint8), pairs=pairs, cpl=cpl,
            rowptr=np.ascontiguousarray(desc.cpl_rowptr, dtype=np.int64),
            f_a=np.ascontiguousarray(desc.f_a, dtype=np.float64), f_b=np.ascontiguousarray(desc.f_b, dtype=np.float64),
            hh=hh, hh_rowptr=hh_rowptr, ring=ring, ring_rowptr=ring_rowptr)
        h = self._host
        prob = Problem(int(desc.n_occ), P, ncpl, h["somo"].ctypes.data, h["pairs"].ctypes.data, h["rowptr"].ctypes.data,
                       h["cpl"].ctypes.data, h["f_a"].ctypes.data, h["f_b"].ctypes.data, int(desc.n_B), int(desc.n_T),
                       int(desc.n_K), int(len(desc.eps_a)), int(desc.n_S), nhh, h["hh_rowptr"].ctypes.data,
                       h["hh"].ctypes.data, nring, h["ring_rowptr"].ctypes.data, h["ring"].ctypes.data,
                       int(getattr(desc, "n_Rg", 0) or 0) if nring > 0 else 0)
        self._dev = [B, S, K, eps_a, eps_b, ring_ints]
        for t in self._dev:
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()):
                raise ValueError("inputs must be contiguous float64 CUDA tensors")
        inp = Inputs(B.data_ptr(), S.data_ptr() if S is not None else None, K.data_ptr(), eps_a.data_ptr(),
                     eps_b.data_ptr(), ring_ints.data_ptr() if ring_ints is not None else None)
        prec = _PREC[precision] if isinstance(precision, str) else int(precision)
        flags = ((FLAG_GENERAL_T if general_T else 0) | (FLAG_QUADRATIC if quadratic else 0)
                 | (FLAG_QUADRATIC_OCC if quadratic_occ else 0))
        opt = Options(prec, diis_max, diis_start, n_workers, int(items_per_wave), flags)
        self.precision = prec
        self.n_T, self.n_B, self.n_pairs = int(desc.n_T), int(desc.n_B), P
        self.n_blocks = int(sum(bin(int(b)).count("1") for b in desc.blocks))
        self._h = C.c_void_p()
        _check(L.dlpno_plan_create(C.byref(prob), C.byref(inp), C.byref(opt), _stream(), C.byref(self._h)))

    # ------------------------------------------------------------------ calls
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().dlpno_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, n):
        import torch
        return torch.empty(max(n, 1), dtype=torch.float64, device="cuda")

    def residual(self, T, R=None):
        R = self._new(self.n_T) if R is None else R
        _check(lib().dlpno_residual(self._h, _ptr(T), _ptr(R), _stream()))
        return R

    def residual_noalloc(self, T, R):
        """dlpno_residual_noalloc: R = residual(T) with the library's static
        scratch as workspace; the caller provides R (nothing is allocated)."""
        _check(lib().dlpno_residual_noalloc(self._h, _ptr(T), _ptr(R), _stream()))
        return R

    def update(self, T, R, T_out=None):
        T_out = self._new(self.n_T) if T_out is None else T_out
        e_pair = self._new(4 * self.n_pairs)
        e_tot = self._new(1)
        _check(lib().dlpno_update(self._h, _ptr(T), _ptr(R), _ptr(T_out), _ptr(e_pair), _ptr(e_tot), _stream()))
        return T_out, e_pair, e_tot

    def f12_energy(self, T, W, scalars, e_pair=None, e_total=None):
        """F12 pair energies with amplitudes T: W (amplitude layout) and
        scalars ([n_blocks, 6]: V, V', B1..B4) are device float64 tensors."""
        e_pair = self._new(4 * self.n_pairs) if e_pair is None else e_pair
        e_total = self._new(1) if e_total is None else e_total
        import torch
        for t in (T, W, scalars):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("T, W and scalars must be contiguous float64 CUDA tensors")
        if T.numel() < self.n_T or W.numel() < self.n_T or scalars.numel() < 6 * self.n_blocks:
            raise ValueError("T and W need n_T doubles, scalars 6 per stored block")
        _check(lib().dlpno_f12_energy(self._h, _ptr(T), _ptr(W), _ptr(scalars), _ptr(e_pair), _ptr(e_total),
                                      _stream()))
        return e_pair, e_total

    def iterate(self, n, T, R=None, e_pair=None, e_total=None, rmax=None):
        R = self._new(self.n_T) if R is None else R
        e_pair = self._new(4 * self.n_pairs) if e_pair is None else e_pair
        e_total = self._new(1) if e_total is None else e_total
        rmax = self._new(1) if rmax is None else rmax
        _check(lib().dlpno_iterate(self._h, int(n), _ptr(T), _ptr(R), _ptr(e_pair), _ptr(e_total), _ptr(rmax),
                                   _stream()))
        return R, e_pair, e_total, rmax

    def solve(self, max_iter, T, tol_r=1e-9, tol_e=1e-10, R=None, e_pair=None, e_total=None, rmax=None):
        """dlpno_solve: iterate to convergence.  Returns (R, e_pair, e_total,
        max|R|, iterations run); raises DlpnoError (status -6) when it does not
        converge in max_iter iterations or diverges."""
        R = self._new(self.n_T) if R is None else R
        e_pair = self._new(4 * self.n_pairs) if e_pair is None else e_pair
        e_total = self._new(1) if e_total is None else e_total
        rmax = self._new(1) if rmax is None else rmax
        n = C.c_int32()
        _check(lib().dlpno_solve(self._h, int(max_iter), float(tol_r), float(tol_e), _ptr(T), _ptr(R), _ptr(e_pair),
                                 _ptr(e_total), _ptr(rmax), C.byref(n), _stream()))
        return R, e_pair, e_total, rmax, n.value

    def checkpoint(self, T):
        """The iteration state (T, DIIS and energy histories) as a host byte array."""
        size = C.c_size_t()
        _check(lib().dlpno_checkpoint_size(self._h, C.byref(size)))
        buf = np.empty(size.value, dtype=np.uint8)
        _check(lib().dlpno_checkpoint_save(self._h, _ptr(T), buf.ctypes.data_as(C.c_void_p), _stream()))
        return buf

    def restore(self, T, buf):
        """Loads a checkpoint into this plan and the device amplitudes T."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib().dlpno_checkpoint_load(self._h, _ptr(T), buf.ctypes.data_as(C.c_void_p), _stream()))

    def reset(self):
        _check(lib().dlpno_reset(self._h, _stream()))

    def history(self, n=4096):
        E = np.zeros(n)
        Rm = np.zeros(n)
        k = lib().dlpno_history(self._h, E.ctypes.data_as(C.POINTER(C.c_double)),
                                Rm.ctypes.data_as(C.POINTER(C.c_double)), n)
        return E[:k], Rm[:k]

    def vjp(self, T, G, dT=None, dB=None, want_dB=True):
        dT = self._new(self.n_T) if dT is None else dT
        if want_dB and dB is None:
            dB = self._new(self.n_B)
        _check(lib().dlpno_residual_vjp(self._h, _ptr(T), _ptr(G), _ptr(dT), _ptr(dB) if want_dB else None,
                                        _stream()))
        return dT, (dB if want_dB else None)

    def solve_mixed(self, n_outer, n_inner, T, R=None, e_pair=None, e_total=None, rmax=None):
        R = self._new(self.n_T) if R is None else R
        e_pair = self._new(4 * self.n_pairs) if e_pair is None else e_pair
        e_total = self._new(1) if e_total is None else e_total
        rmax = self._new(1) if rmax is None else rmax
        _check(lib().dlpno_solve_mixed(self._h, int(n_outer), int(n_inner), _ptr(T), _ptr(R), _ptr(e_pair),
                                       _ptr(e_total), _ptr(rmax), _stream()))
        return R, e_pair, e_total, rmax

    def diis_state(self):
        """(vectors kept, vectors dropped since the reset, coefficients oldest -> newest)."""
        cnt, drops = C.c_int32(), C.c_int32()
        coef = (C.c_double * 8)()
        _check(lib().dlpno_diis_state(self._h, C.byref(cnt), C.byref(drops), coef, _stream()))
        return cnt.value, drops.value, np.array(coef[:cnt.value])

    def flop_count(self):
        a, b = C.c_double(), C.c_double()
        _check(lib().dlpno_flop_count(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def autotune(self, T, R=None):
        R = self._new(self.n_T) if R is None else R
        _check(lib().dlpno_autotune(self._h, _ptr(T), _ptr(R), _stream()))

    def autotune_cached(self, T, path, R=None):
        """dlpno_autotune_cached: the tuned schedule from the JSON cache `path`
        (True) or tuned now and stored there (False)."""
        R = self._new(self.n_T) if R is None else R
        hit = C.c_int32()
        _check(lib().dlpno_autotune_cached(self._h, _ptr(T), _ptr(R), os.fsencode(path), C.byref(hit), _stream()))
        return bool(hit.value)

    def set_profiling(self, on=True):
        _check(lib().dlpno_set_profiling(self._h, 1 if on else 0))

    def phase_times(self):
        ms = (C.c_double * 11)()
        n = (C.c_int64 * 11)()
        _check(lib().dlpno_phase_times(self._h, ms, n, 11))
        return list(ms), list(n)

    def ring_flop_count(self):
        """(flops, contractions) of the ring/exchange term per residual."""
        f = C.c_double()
        k = C.c_int64()
        _check(lib().dlpno_ring_flop_count(self._h, C.byref(f), C.byref(k)))
        return f.value, k.value

    def info(self):
        return lib().dlpno_plan_info(self._h).decode()


class PnoPlan:
    """PNO construction over device-resident inputs (dlpno_pno_*).

    pairs: numpy array of workload.pno.PNO_PAIR_DTYPE (the dlpno_pno_pair
    layout); n_X, n_F, n_C, n_v: buffer sizes in doubles."""

    def __init__(self, pairs, n_X, n_F, n_C, n_v):
        pairs = np.ascontiguousarray(pairs)
        if pairs.dtype.itemsize != 48:
            raise ValueError("pairs must use the 48-byte dlpno_pno_pair layout")
        self.n_pairs, self.n_C, self.n_v = len(pairs), int(n_C), int(n_v)
        self._pairs = pairs
        self._h = C.c_void_p()
        _check(lib().dlpno_pno_plan_create(pairs.ctypes.data_as(C.c_void_p), self.n_pairs, int(n_X), int(n_F),
                                           self.n_C, self.n_v, C.byref(self._h)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().dlpno_pno_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build(self, X, F, t_cut, occ=None, eps=None, Cout=None, n_kept=None, sweeps=None, want_sweeps=False):
        """Returns (occ, eps, C, n_kept, sweeps) as device tensors (sweeps is
        None unless requested)."""
        import torch
        dev = F.device
        f64 = dict(dtype=torch.float64, device=dev)
        occ = torch.empty(max(self.n_v, 1), **f64) if occ is None else occ
        eps = torch.empty(max(self.n_v, 1), **f64) if eps is None else eps
        Cout = torch.empty(max(self.n_C, 1), **f64) if Cout is None else Cout
        n_kept = torch.empty(max(self.n_pairs, 1), dtype=torch.int32, device=dev) if n_kept is None else n_kept
        if sweeps is None and want_sweeps:
            sweeps = torch.empty(max(2 * self.n_pairs, 1), dtype=torch.int32, device=dev)
        _check(lib().dlpno_pno_build(self._h, _ptr(X), _ptr(F), float(t_cut), _ptr(occ), _ptr(eps), _ptr(Cout),
                                     _ptr(n_kept), _ptr(sweeps), _stream()))
        return occ, eps, Cout, n_kept, sweeps

    def overlap_prepare(self, n_kept, rowptr, src, off_S, n_S):
        """Coupling list of overlap(): host arrays (n_kept as returned by
        build, copied to the host)."""
        self._cpl = [np.ascontiguousarray(n_kept, dtype=np.int32), np.ascontiguousarray(rowptr, dtype=np.int64),
                     np.ascontiguousarray(src, dtype=np.int32), np.ascontiguousarray(off_S, dtype=np.int64)]
        self.n_S = int(n_S)
        _check(lib().dlpno_pno_overlap_prepare(self._h, *[a.ctypes.data_as(C.c_void_p) for a in self._cpl],
                                               self.n_S))

    def overlap(self, Cmat, S=None):
        import torch
        S = torch.empty(max(self.n_S, 1), dtype=torch.float64, device=Cmat.device) if S is None else S
        _check(lib().dlpno_pno_overlap(self._h, _ptr(Cmat), _ptr(S), _stream()))
        return S
