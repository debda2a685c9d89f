"""Thin ctypes binding of ``libptm.so`` (C ABI in include/ptm.h).

Names follow the C functions.  This module only marshals arguments: every
step of the classification runs in the library's HIP kernels.  PyTorch is
used for device memory (``Classifier`` allocates output tensors and passes
their ``data_ptr()``).  If the library is missing the import of the
library fails loudly; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libptm.so")

PTM_OK, PTM_E_INVALID, PTM_E_NOMEM, PTM_E_DEVICE, PTM_E_BOX, PTM_E_TOO_LARGE, PTM_E_BUSY, PTM_E_TIMEOUT = range(8)
PTM_FP64, PTM_FP32_MIXED = 0, 1
PTM_SC, PTM_FCC, PTM_HCP, PTM_ICO, PTM_BCC = 1, 2, 4, 8, 16
PTM_ALL = 0x1F
PTM_F_HOST_POINTERS = 1
PTM_F_PROFILE = 2
PTM_F_TOPOLOGICAL = 4
PTM_F_FULL_RULE = 8
PTM_F_PERSISTENT = 16
STAGE_NAMES = ("bounds", "bin", "knn", "topo", "match")
TYPE_NAMES = ("NONE", "SC", "FCC", "HCP", "ICO", "BCC")
ALLOY_NAMES = ("NONE", "A1", "L1_0", "L1_2_maj", "L1_2_min", "FCC_other", "A2", "B2", "BCC_other")


class ptm_config(C.Structure):
    _fields_ = [("device", C.c_int), ("precision", C.c_int), ("hip_stream", C.c_void_p),
                ("hbm_budget_bytes", C.c_uint64), ("flags", C.c_uint32)]


OUTPUT_FIELDS = ("type", "alloy", "rmsd", "scale", "quat", "neighbours", "strain", "knn",
                 "vm_strain", "strain_residual", "nn_distance", "quat_fz", "best_type")


class ptm_outputs(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in OUTPUT_FIELDS]


class ptm_frame_stats(C.Structure):
    _fields_ = [("submit_time_us", C.c_double), ("start_time_us", C.c_double),
                ("complete_time_us", C.c_double), ("n_atoms", C.c_int64), ("scratch_bytes", C.c_uint64)]


class PTMError(RuntimeError):
    def __init__(self, status, message=""):
        self.status = status
        super().__init__(f"{ptm_status_string(status)} ({status}): {message}")


_lib = None


def lib():
    """Load libptm.so (built by paper_1603_05143_amd.build_lib)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        # PyTorch ships its own HIP runtime under the soname the library
        # links against.  Loaded after torch, the library binds to torch's
        # copy, so device pointers and streams from torch are valid in it;
        # loaded first, torch would bring a second runtime into the process
        # and the library's calls would fail.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.ptm_create.argtypes = [C.POINTER(ptm_config), C.POINTER(vp)]
        L.ptm_create.restype = C.c_int
        L.ptm_classify.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_uint32, C.c_double, C.POINTER(ptm_outputs)]
        L.ptm_classify.restype = C.c_int
        L.ptm_classify_noalloc.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_uint32, C.c_double,
                                           C.POINTER(ptm_outputs)]
        L.ptm_classify_noalloc.restype = C.c_int
        L.ptm_submit.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_uint32, C.c_double, C.POINTER(ptm_outputs),
                                 C.POINTER(C.c_uint64)]
        L.ptm_submit.restype = C.c_int
        L.ptm_wait.argtypes = [vp, C.c_uint64, C.c_int64, C.POINTER(ptm_frame_stats)]
        L.ptm_wait.restype = C.c_int
        L.ptm_destroy.argtypes = [vp]
        L.ptm_destroy.restype = None
        L.ptm_status_string.argtypes = [C.c_int]
        L.ptm_status_string.restype = C.c_char_p
        L.ptm_last_error.argtypes = [vp]
        L.ptm_last_error.restype = C.c_char_p
        L.ptm_template_info.argtypes = [C.c_int, C.POINTER(C.c_int64)]
        L.ptm_template_info.restype = C.c_int
        L.ptm_stage_times.argtypes = [vp, C.POINTER(C.c_double), C.c_int]
        L.ptm_stage_times.restype = C.c_int
        L.ptm_frame_info.argtypes = [vp, C.POINTER(C.c_int64), C.c_int]
        L.ptm_frame_info.restype = C.c_int
        L.ptm_misorientation.argtypes = [vp, vp, vp, vp, C.c_int64, vp]
        L.ptm_misorientation.restype = C.c_int
        L.ptm_apply_cutoff.argtypes = [vp, vp, vp, C.c_int64, C.c_double, vp]
        L.ptm_apply_cutoff.restype = C.c_int
        L.ptm_rmsd_histogram.argtypes = [vp, vp, vp, C.c_int64, C.c_int, C.c_double, C.POINTER(C.c_int64)]
        L.ptm_rmsd_histogram.restype = C.c_int
        _lib = L
    return _lib


# ---- same names as the C ABI --------------------------------------------
def ptm_status_string(status: int) -> str:
    return lib().ptm_status_string(status).decode()


def ptm_last_error(ctx) -> str:
    return lib().ptm_last_error(ctx).decode()


def ptm_create(device=0, precision=PTM_FP64, hip_stream=None, hbm_budget_bytes=0, flags=0):
    cfg = ptm_config(device, precision, hip_stream, hbm_budget_bytes, flags)
    ctx = C.c_void_p()
    st = lib().ptm_create(C.byref(cfg), C.byref(ctx))
    if st != PTM_OK:
        raise PTMError(st, "ptm_create")
    return ctx


def ptm_destroy(ctx) -> None:
    lib().ptm_destroy(ctx)


def ptm_classify(ctx, positions_ptr, species_ptr, box, n_atoms, template_mask, rmsd_cutoff, outputs):
    bx = (C.c_double * 3)(*[float(b) for b in box])
    return lib().ptm_classify(ctx, positions_ptr, species_ptr, bx, int(n_atoms), int(template_mask),
                              float(rmsd_cutoff), C.byref(outputs))


def ptm_classify_noalloc(ctx, positions_ptr, species_ptr, box, n_atoms, template_mask, rmsd_cutoff, outputs):
    bx = (C.c_double * 3)(*[float(b) for b in box])
    return lib().ptm_classify_noalloc(ctx, positions_ptr, species_ptr, bx, int(n_atoms), int(template_mask),
                                      float(rmsd_cutoff), C.byref(outputs))


PTM_NOALLOC_MAX_ATOMS = 65536


def ptm_submit(ctx, positions_ptr, species_ptr, box, n_atoms, template_mask, rmsd_cutoff, outputs):
    bx = (C.c_double * 3)(*[float(b) for b in box])
    t = C.c_uint64()
    st = lib().ptm_submit(ctx, positions_ptr, species_ptr, bx, int(n_atoms), int(template_mask),
                          float(rmsd_cutoff), C.byref(outputs), C.byref(t))
    return st, t.value


def ptm_wait(ctx, ticket, timeout_us=-1):
    s = ptm_frame_stats()
    st = lib().ptm_wait(ctx, C.c_uint64(ticket), int(timeout_us), C.byref(s))
    return st, s


def ptm_stage_times(ctx):
    """Stage times (ms) of the last ptm_classify on a PTM_F_PROFILE context."""
    ms = (C.c_double * len(STAGE_NAMES))()
    st = lib().ptm_stage_times(ctx, ms, len(STAGE_NAMES))
    if st != PTM_OK:
        raise PTMError(st, "ptm_stage_times")
    return dict(zip(STAGE_NAMES, list(ms)))


INFO_NAMES = ("cells", "knn_exact", "pairs", "decide_full")


def ptm_frame_info(ctx):
    """Work counts of the last ptm_classify on a PTM_F_PROFILE context."""
    info = (C.c_int64 * len(INFO_NAMES))()
    st = lib().ptm_frame_info(ctx, info, len(INFO_NAMES))
    if st != PTM_OK:
        raise PTMError(st, "ptm_frame_info")
    return dict(zip(INFO_NAMES, list(info)))


def ptm_misorientation(ctx, type_ptr, q1_ptr, q2_ptr, n, angle_ptr):
    return lib().ptm_misorientation(ctx, type_ptr, q1_ptr, q2_ptr, int(n), angle_ptr)


def ptm_apply_cutoff(ctx, best_type_ptr, rmsd_ptr, n, cutoff, type_ptr):
    return lib().ptm_apply_cutoff(ctx, best_type_ptr, rmsd_ptr, int(n), float(cutoff), type_ptr)


def ptm_rmsd_histogram(ctx, best_type_ptr, rmsd_ptr, n, nbins, rmax):
    """Returns (status, counts[6][nbins] as a list of lists)."""
    counts = (C.c_int64 * (6 * int(nbins)))()
    st = lib().ptm_rmsd_histogram(ctx, best_type_ptr, rmsd_ptr, int(n), int(nbins), float(rmax), counts)
    return st, [list(counts[t * nbins:(t + 1) * nbins]) for t in range(6)]


def ptm_template_info(t: int):
    info = (C.c_int64 * 5)()
    st = lib().ptm_template_info(t, info)
    if st != PTM_OK:
        raise PTMError(st, "ptm_template_info")
    return {"k": info[0], "group_order": info[1], "triangulations": info[2], "codes": info[3],
            "candidates": info[4]}


# ---- convenience wrapper over torch device tensors ------------------------
class Classifier:
    """Owns a context; classifies torch tensors resident on the GPU."""

    def __init__(self, device: int = 0, precision: int = PTM_FP64, hbm_budget_bytes: int = 0,
                 topological: bool = False, flags: int = 0):
        import torch
        self.device = device
        self.precision = precision
        self.topological = topological
        # the library runs on a torch stream of its own, which waits for the
        # caller's current stream before every call (inputs written by torch
        # kernels still in flight; output blocks the caching allocator handed
        # out on that stream)
        self.stream = torch.cuda.Stream(device=device)
        self.ctx = ptm_create(device, precision, self.stream.cuda_stream, hbm_budget_bytes,
                              flags | (PTM_F_TOPOLOGICAL if topological else 0))

    def close(self):
        if self.ctx is not None:
            ptm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def alloc_outputs(n: int, device: str, knn: bool = False, derived: bool = False, best_type: bool = False):
        import torch
        out = {
            "type": torch.empty(n, dtype=torch.int8, device=device),
            "alloy": torch.empty(n, dtype=torch.int8, device=device),
            "rmsd": torch.empty(n, dtype=torch.float64, device=device),
            "scale": torch.empty(n, dtype=torch.float64, device=device),
            "quat": torch.empty((n, 4), dtype=torch.float64, device=device),
            "neighbours": torch.empty((n, 14), dtype=torch.int32, device=device),
            "strain": torch.empty((n, 9), dtype=torch.float64, device=device),
        }
        if knn:
            out["knn"] = torch.empty((n, 14), dtype=torch.int32, device=device)
        if derived:
            for k in ("vm_strain", "strain_residual", "nn_distance"):
                out[k] = torch.empty(n, dtype=torch.float64, device=device)
            out["quat_fz"] = torch.empty((n, 4), dtype=torch.float64, device=device)
        if derived or best_type:
            out["best_type"] = torch.empty(n, dtype=torch.int8, device=device)
        return out

    @staticmethod
    def outputs_struct(out) -> ptm_outputs:
        def p(k):
            t = out.get(k)
            return None if t is None else t.data_ptr()
        return ptm_outputs(*[p(k) for k in OUTPUT_FIELDS])

    def classify(self, positions, box, species=None, mask=PTM_ALL, cutoff=float("inf"), out=None, knn=False,
                 derived=False, best_type=False):
        """positions: (n,3) float64 CUDA tensor; returns dict of output tensors."""
        import torch
        assert positions.is_cuda and positions.dtype == torch.float64 and positions.is_contiguous()
        n = positions.shape[0]
        if out is None:
            out = self.alloc_outputs(n, positions.device, knn, derived, best_type)
        sp = None
        if species is not None:
            assert species.is_cuda and species.dtype == torch.int8 and species.is_contiguous()
            sp = species.data_ptr()
        self.stream.wait_stream(torch.cuda.current_stream(positions.device))
        st = ptm_classify(self.ctx, positions.data_ptr() if n else None, sp, box, n, mask, cutoff,
                          self.outputs_struct(out))
        if st != PTM_OK:
            raise PTMError(st, ptm_last_error(self.ctx))
        return out

    def apply_cutoff(self, out, cutoff):
        """Types under a new RMSD cut-off from the outputs of a classify call
        that kept best_type; returns a new int8 tensor."""
        import torch
        n = out["rmsd"].shape[0]
        t = torch.empty(n, dtype=torch.int8, device=out["rmsd"].device)
        self.stream.wait_stream(torch.cuda.current_stream(t.device))
        st = ptm_apply_cutoff(self.ctx, out["best_type"].data_ptr() if n else None,
                              out["rmsd"].data_ptr() if n else None, n, cutoff, t.data_ptr() if n else None)
        if st != PTM_OK:
            raise PTMError(st, ptm_last_error(self.ctx))
        return t

    def rmsd_histogram(self, out, nbins, rmax):
        """Per-type RMSD histograms (6 x nbins int64 numpy array)."""
        import numpy as np
        import torch
        n = out["rmsd"].shape[0]
        self.stream.wait_stream(torch.cuda.current_stream(out["rmsd"].device))
        st, counts = ptm_rmsd_histogram(self.ctx, out["best_type"].data_ptr() if n else None,
                                        out["rmsd"].data_ptr() if n else None, n, nbins, rmax)
        if st != PTM_OK:
            raise PTMError(st, ptm_last_error(self.ctx))
        return np.array(counts, dtype=np.int64)
