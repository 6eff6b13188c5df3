"""ctypes binding of libsn.so (argument marshalling only; every step of the
evaluation runs in the library's HIP kernels).

torch is imported first so that the process has a single HIP runtime and
the library can work on torch's device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (HIP runtime first; device tensors for the *_device entry points)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsn.so")

SN_OK, SN_EINVAL, SN_ENOMEM, SN_EHIP, SN_EUNSUPPORTED, SN_EBUSY = 0, -1, -2, -3, -4, -5
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}


class SNError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libsn error {status}: {msg}")
        self.status = status


class ModelInfo(C.Structure):
    _fields_ = [
        ("n_layers", C.c_int), ("l_max", C.c_int), ("l_sh", C.c_int), ("muls", C.c_int * 4),
        ("n_basis", C.c_int), ("hidden", C.c_int), ("n_species", C.c_int),
        ("species_z", C.c_int * 128), ("r_cut", C.c_double), ("k_avg", C.c_double),
        ("sigma", C.c_double), ("n_params", C.c_int64),
    ]


class Request(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("pos", C.c_void_p), ("Z", C.c_void_p), ("cell", C.c_void_p),
        ("atom_energy", C.c_void_p), ("forces", C.c_void_p),
    ]


class Result(C.Structure):
    _fields_ = [
        ("ticket", C.c_uint64), ("status", C.c_int), ("batch_structures", C.c_int),
        ("batch_atoms", C.c_int64), ("energy", C.c_double), ("virial", C.c_double * 9),
        ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
    ]


class Batch(C.Structure):
    """sn_batch_t: a packed batch of structures in device memory."""
    _fields_ = [
        ("n_structures", C.c_int32), ("offsets", C.c_void_p), ("cells", C.c_void_p),
        ("d_pos", C.c_void_p), ("d_Z", C.c_void_p),
    ]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)


class Allocator(C.Structure):
    """sn_allocator_t: device allocations of a context through caller callbacks."""
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "sn_strerror": (C.c_char_p, [C.c_int]),
    "sn_last_error": (C.c_char_p, [C.c_void_p]),
    "sn_model_load": (C.c_int, [C.c_char_p, C.POINTER(C.c_void_p)]),
    "sn_model_free": (None, [C.c_void_p]),
    "sn_model_info": (C.c_int, [C.c_void_p, C.POINTER(ModelInfo)]),
    "sn_cg_table": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_void_p]),
    "sn_ctx_create": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_size_t, C.c_int, C.c_double,
                                C.POINTER(Allocator), C.POINTER(C.c_void_p)]),
    "sn_ctx_free": (None, [C.c_void_p]),
    "sn_compute": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sn_compute_noalloc": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sn_compute_batch": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sn_forward_device": (C.c_int, [C.c_void_p, C.POINTER(Batch), C.c_void_p, C.c_void_p]),
    "sn_backward_device": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sn_ctx_synchronize": (C.c_int, [C.c_void_p]),
    "sn_ctx_set_training": (C.c_int, [C.c_void_p, C.c_int]),
    "sn_backward_train_device": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p]),
    "sn_train_loss_grad": (C.c_int, [C.c_void_p, C.POINTER(Batch), C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.POINTER(C.c_double), C.c_void_p]),
    "sn_model_tensor": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_char_p),
                                  C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "sn_huber_energy_loss": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                       C.POINTER(C.c_double), C.c_void_p]),
    "sn_ctx_graph_size": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64)]),
    "sn_ctx_evaluated_edges": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "sn_ctx_set_edge_compaction": (C.c_int, [C.c_void_p, C.c_int]),
    "sn_ctx_pair_count": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "sn_ctx_set_graph_reuse": (C.c_int, [C.c_void_p, C.c_int]),
    "sn_ctx_set_domains": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int]),
    "sn_ctx_set_capture": (C.c_int, [C.c_void_p, C.c_int]),
    "sn_md_verlet": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_double, C.c_int]),
    "sn_md_nh_half": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_double,
                                C.c_double, C.c_double, C.c_double, C.c_void_p]),
    "sn_md_max_displacement": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                         C.POINTER(C.c_double)]),
    "sn_ctx_graph": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p]),
    "sn_ctx_memory": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "sn_server_create": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_size_t, C.c_int64,
                                   C.c_int, C.POINTER(C.c_void_p)]),
    "sn_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "sn_server_warmup": (C.c_int, [C.c_void_p, C.POINTER(Request)]),
    "sn_server_poll": (C.c_int, [C.c_void_p, C.POINTER(Result), C.c_int, C.c_int,
                                 C.POINTER(C.c_int)]),
    "sn_server_pending": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "sn_server_free": (None, [C.c_void_p]),
    "sn_ctx_timings": (C.c_int, [C.c_void_p, C.POINTER(C.c_char_p), C.c_void_p,
                                 C.POINTER(C.c_int)]),
}

EXPORTED = tuple(_SIGS)


def lib():
    """The loaded library; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status, ctx=None):
    if status != SN_OK:
        msg = lib().sn_last_error(ctx).decode()
        raise SNError(status, f"{lib().sn_strerror(status).decode()}: {msg}")


def ptr(a) -> C.c_void_p:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    if isinstance(a, torch.Tensor):
        return C.c_void_p(a.data_ptr())
    raise TypeError(type(a))
