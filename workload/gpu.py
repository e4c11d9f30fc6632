"""Generate a workload's large fields directly in device memory (torch tensors).

Uses the HIP build of the same counter-based generator as workload.philox, so
every element is bit-identical to what the host generator produces.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libdlpno_gen.so")
        if not os.path.exists(path):
            raise ImportError("workload generator library not built: %s (run __graft_entry__.build())" % path)
        L = ctypes.CDLL(path)
        L.dlpno_gen_segments.restype = ctypes.c_int
        L.dlpno_gen_segments.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p,
                                         ctypes.c_void_p]
        _LIB = L
    return _LIB


def fill(out, segs, seed, stream=None, chunk=1 << 20):
    """Fill the float64 CUDA tensor `out` with the generated segments."""
    import torch
    if len(segs) == 0:
        return out
    st = torch.cuda.current_stream() if stream is None else stream
    for a in range(0, len(segs), chunk):
        part = np.ascontiguousarray(segs[a:a + chunk])
        d = torch.from_numpy(part.view(np.uint8).copy()).to(out.device)
        rc = lib().dlpno_gen_segments(ctypes.c_void_p(d.data_ptr()), len(part), int(seed),
                                      ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.cuda_stream))
        if rc != 0:
            raise RuntimeError("generator launch failed (hipError %d)" % rc)
        st.synchronize()
        del d
    return out


def device_fields(prob, device="cuda", fields=("B", "S", "K", "T"), dtype=None):
    """Allocate and generate the requested flat fields on the GPU."""
    import torch
    out = {}
    sizes = {"B": prob.n_B, "S": prob.n_S, "K": prob.n_K, "T": prob.n_T, "W": prob.n_T, "Rg": prob.n_Rg}
    for f in fields:
        t = torch.empty(max(sizes[f], 1), dtype=torch.float64, device=device)
        if f == "S" and prob.S_host is not None:
            t[:prob.n_S].copy_(torch.from_numpy(prob.S_host))
        else:
            t.zero_()
            fill(t, prob.segs[f], prob.seed)
        out[f] = t
    return out


def device_pno_fields(prob, device="cuda"):
    """X and F of a PNO workload (workload.pno) generated on the GPU."""
    import torch
    out = {}
    for f, n in (("X", prob.n_X), ("F", prob.n_F)):
        t = torch.zeros(max(n, 1), dtype=torch.float64, device=device)
        fill(t, prob.segs[f], prob.seed)
        out[f] = t
    return out
