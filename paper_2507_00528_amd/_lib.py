"""ctypes view of libnep's C ABI (include/nep.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnep.so")

c_float_p = C.POINTER(C.c_float)
c_int32_p = C.POINTER(C.c_int32)


class NepModel(C.Structure):
    _fields_ = [("n_types", C.c_int32), ("n_rad", C.c_int32), ("n_ang", C.c_int32), ("k_rad", C.c_int32),
                ("k_ang", C.c_int32), ("l3", C.c_int32), ("l4", C.c_int32), ("l5", C.c_int32),
                ("hidden", C.c_int32), ("rc_rad", C.c_float), ("rc_ang", C.c_float),
                ("cap_rad", C.c_int32), ("cap_ang", C.c_int32)]


class NepBatch(C.Structure):
    _fields_ = [("n_struct", C.c_int32), ("n_atom", C.c_int32), ("atom_offset", C.c_void_p),
                ("box", C.c_void_p), ("pos", C.c_void_p), ("type", C.c_void_p), ("tilt", C.c_void_p),
                ("max_atoms", C.c_int32)]


class NepNeighbors(C.Structure):
    _fields_ = [("idx_rad", C.c_void_p), ("cnt_rad", C.c_void_p), ("idx_ang", C.c_void_p), ("cnt_ang", C.c_void_p)]


class NepLabels(C.Structure):
    _fields_ = [("energy", C.c_void_p), ("force", C.c_void_p), ("virial", C.c_void_p)]


class NepAdamConfig(C.Structure):
    _fields_ = [("lr_start", C.c_float), ("lr_stop", C.c_float), ("n_warmup", C.c_int64), ("n_total", C.c_int64),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


class NepTuning(C.Structure):
    _fields_ = [("persistent", C.c_int32), ("outer_blocks_w", C.c_int32), ("outer_blocks_c", C.c_int32),
                ("reduce_chunks", C.c_int32), ("cell_min_atoms", C.c_int32), ("gather_lanes", C.c_int32),
                ("forward_waves", C.c_int32), ("adjoint_waves", C.c_int32),
                ("reverse_branch", C.c_int32)]


P = C.POINTER
VP = C.c_void_p
I32 = C.c_int32
F32 = C.c_float

# (name, restype, argtypes) of every exported entry point of include/nep.h
SIGNATURES = [
    ("nep_param_count", C.c_int64, [P(NepModel)]),
    ("nep_descriptor_count", I32, [P(NepModel)]),
    ("nep_model_supported", C.c_int, [P(NepModel)]),
    ("nep_workspace_bytes", C.c_int, [P(NepModel), I32, I32, P(C.c_size_t)]),
    ("nep_build_neighbors", C.c_int, [P(NepModel), P(NepBatch), P(NepNeighbors), VP, VP, VP]),
    ("nep_descriptors", C.c_int, [P(NepModel), P(NepBatch), P(NepNeighbors), VP, VP, VP, VP]),
    ("nep_energy_force_virial", C.c_int, [P(NepModel), P(NepBatch), P(NepNeighbors), VP, VP, VP, VP, VP, VP, VP]),
    ("nep_vjp", C.c_int, [P(NepModel), P(NepBatch), P(NepNeighbors), VP, VP, VP, VP, VP, VP, VP]),
    ("nep_loss_grad", C.c_int, [P(NepModel), P(NepBatch), P(NepNeighbors), VP, P(NepLabels), P(F32 * 3),
                                VP, VP, VP, VP, VP, VP, VP, VP]),
    ("nep_loss_grad_noalloc", C.c_int, [P(NepModel), P(NepBatch), P(NepNeighbors), VP, P(NepLabels),
                                        P(F32 * 3), VP, VP, VP, VP, VP, VP, VP]),
    ("nep_adam_step", C.c_int, [C.c_int64, VP, VP, VP, VP, F32, F32, F32, F32, I32, VP]),
    ("nep_lr_schedule", F32, [C.c_int64, F32, F32, C.c_int64, C.c_int64]),
    ("nep_md_step", C.c_int, [P(NepModel), P(NepBatch), VP, P(NepNeighbors), VP, VP, VP, VP, F32, I32, VP, VP,
                              VP, VP, VP]),
    ("nep_train_step_graph_create", C.c_int, [P(NepModel), P(NepBatch), P(NepNeighbors), P(NepLabels),
                                              P(F32 * 3), VP, VP, VP, VP, VP, VP, P(NepAdamConfig), VP, VP, I32,
                                              VP, P(VP)]),
    ("nep_train_step_graph_create_tuned", C.c_int, [P(NepModel), P(NepBatch), P(NepNeighbors), P(NepLabels),
                                                    P(F32 * 3), VP, VP, VP, VP, VP, VP, P(NepAdamConfig), VP, VP,
                                                    I32, P(NepTuning), VP, P(VP)]),
    ("nep_train_step_graph_launch", C.c_int, [VP, VP]),
    ("nep_train_step_graph_destroy", C.c_int, [VP]),
    ("nep_profile_loss_grad", C.c_int, [P(NepModel), P(NepBatch), P(NepNeighbors), VP, P(NepLabels), P(F32 * 3),
                                        VP, VP, VP, VP, VP, P(F32), P(C.c_char_p), I32, P(I32)]),
    ("nep_flags_status", C.c_int, [I32]),
    ("nep_status_string", C.c_char_p, [C.c_int]),
]

_lib = None


def load() -> C.CDLL:
    """The built libnep.so; raises when it has not been built (there is no
    fallback implementation)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2507_00528_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
