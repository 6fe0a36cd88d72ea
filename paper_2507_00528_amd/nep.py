"""Python binding of libnep with the names of the C ABI (include/nep.h).

PyTorch supplies device memory and streams; every step of the computation
runs in the library's HIP kernels.  Functions take torch tensors already on
the GPU, check dtypes/shapes, and pass raw pointers plus the current HIP
stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib

NEP_FLAG_NBR_OVERFLOW = 1
NEP_FLAG_NONFINITE = 2
NEP_FLAG_BOX = 4
NEP_FLAG_TYPE = 8
NEP_FLAG_POSITION = 16
NEP_FLAG_STEP = 32


class NEPError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.load().nep_status_string(code).decode()
        super().__init__(f"{where}: {msg} (status {code})")
        self.code = code


def _check(code: int, where: str):
    if code != 0:
        raise NEPError(code, where)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _want(t, dtype, numel, name):
    if t.dtype != dtype or t.numel() != numel:
        raise ValueError(f"{name}: expected {dtype} with {numel} elements, got {t.dtype} {tuple(t.shape)}")


@dataclass
class Model:
    """NEP sizes (counts) plus neighbor capacities; see nep_model."""
    n_types: int
    n_rad: int
    n_ang: int
    k_rad: int
    k_ang: int
    l3: int
    l4: int
    l5: int
    hidden: int
    rc_rad: float
    rc_ang: float
    cap_rad: int = 64
    cap_ang: int = 32

    @classmethod
    def of(cls, sizes, cap_rad=64, cap_ang=32):
        return cls(sizes.n_types, sizes.n_rad, sizes.n_ang, sizes.k_rad, sizes.k_ang, sizes.l3, sizes.l4,
                   sizes.l5, sizes.hidden, float(sizes.rc_rad), float(sizes.rc_ang), cap_rad, cap_ang)

    def c(self):
        return _lib.NepModel(self.n_types, self.n_rad, self.n_ang, self.k_rad, self.k_ang, self.l3, self.l4,
                             self.l5, self.hidden, self.rc_rad, self.rc_ang, self.cap_rad, self.cap_ang)


def param_count(model: Model) -> int:
    v = _lib.load().nep_param_count(C.byref(model.c()))
    _check(int(v) if v < 0 else 0, "nep_param_count")
    return int(v)


def descriptor_count(model: Model) -> int:
    v = _lib.load().nep_descriptor_count(C.byref(model.c()))
    _check(int(v) if v < 0 else 0, "nep_descriptor_count")
    return int(v)


def model_supported(model: Model) -> bool:
    return _lib.load().nep_model_supported(C.byref(model.c())) == 0


def workspace_bytes(model: Model, n_struct: int, n_atom: int) -> int:
    out = C.c_size_t(0)
    _check(_lib.load().nep_workspace_bytes(C.byref(model.c()), n_struct, n_atom, C.byref(out)),
           "nep_workspace_bytes")
    return int(out.value)


class DeviceBatch:
    """Batch arrays on the GPU in the library's layout."""

    def __init__(self, batch, device="cuda"):
        self.n_struct = int(batch.n_struct)
        self.n_atom = int(batch.n_atom)
        self.atom_offset = torch.as_tensor(np.asarray(batch.atom_offset, np.int32), device=device)
        self.box = torch.as_tensor(np.asarray(batch.box, np.float32), device=device)
        self.pos = torch.as_tensor(np.asarray(batch.pos_soa, np.float32), device=device)
        self.type = torch.as_tensor(np.asarray(batch.types, np.int32), device=device)
        # tilts (xy, xz, yz) per structure; None when every cell is orthorhombic
        tilt = getattr(batch, "tilt", None)
        self.tilt = (torch.as_tensor(np.asarray(tilt, np.float32), device=device)
                     if tilt is not None and np.any(np.asarray(tilt) != 0) else None)
        # largest structure: batches of small structures skip the cell-list kernels
        self.max_atoms = int(np.diff(np.asarray(batch.atom_offset)).max()) if self.n_struct else 0

    def c(self):
        return _lib.NepBatch(self.n_struct, self.n_atom, self.atom_offset.data_ptr(), self.box.data_ptr(),
                             self.pos.data_ptr() if self.n_atom else None,
                             self.type.data_ptr() if self.n_atom else None,
                             self.tilt.data_ptr() if self.tilt is not None else None, self.max_atoms)


class Neighbors:
    def __init__(self, model: Model, n_atom: int, device="cuda"):
        n = max(n_atom, 1)
        self.idx_rad = torch.zeros(model.cap_rad * n, dtype=torch.int32, device=device)
        self.cnt_rad = torch.zeros(n, dtype=torch.int32, device=device)
        self.idx_ang = torch.zeros(model.cap_ang * n, dtype=torch.int32, device=device)
        self.cnt_ang = torch.zeros(n, dtype=torch.int32, device=device)

    def c(self):
        return _lib.NepNeighbors(self.idx_rad.data_ptr(), self.cnt_rad.data_ptr(), self.idx_ang.data_ptr(),
                                 self.cnt_ang.data_ptr())


def workspace(model: Model, n_struct: int, n_atom: int, device="cuda") -> torch.Tensor:
    nb = workspace_bytes(model, n_struct, n_atom)
    ws = torch.empty(max(nb, 256) + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + max(nb, 256)]


def build_neighbors(model, batch: DeviceBatch, nbrs: Neighbors, ws, flags, stream=None):
    _want(flags, torch.int32, 1, "flags")
    _check(_lib.load().nep_build_neighbors(C.byref(model.c()), C.byref(batch.c()), C.byref(nbrs.c()), _ptr(ws),
                                           _ptr(flags), _stream(stream)), "nep_build_neighbors")


def descriptors(model, batch, nbrs, params, G, ws, stream=None):
    _want(params, torch.float32, param_count(model), "params")
    _want(G, torch.float32, descriptor_count(model) * batch.n_atom, "G")
    _check(_lib.load().nep_descriptors(C.byref(model.c()), C.byref(batch.c()), C.byref(nbrs.c()), _ptr(params),
                                       _ptr(G), _ptr(ws), _stream(stream)), "nep_descriptors")


def energy_force_virial(model, batch, nbrs, params, ws, e_atom=None, e_struct=None, force=None, virial=None,
                        stream=None):
    _want(params, torch.float32, param_count(model), "params")
    for t, n, name in ((e_atom, batch.n_atom, "e_atom"), (e_struct, batch.n_struct, "e_struct"),
                       (force, 3 * batch.n_atom, "force"), (virial, 6 * batch.n_struct, "virial")):
        if t is not None:
            _want(t, torch.float32, n, name)
    _check(_lib.load().nep_energy_force_virial(C.byref(model.c()), C.byref(batch.c()), C.byref(nbrs.c()),
                                               _ptr(params), _ptr(e_atom), _ptr(e_struct), _ptr(force),
                                               _ptr(virial), _ptr(ws), _stream(stream)), "nep_energy_force_virial")


def vjp(model, batch, nbrs, params, e_bar, f_bar, v_bar, grad, ws, stream=None):
    P = param_count(model)
    _want(params, torch.float32, P, "params")
    _want(grad, torch.float32, P, "grad")
    _want(e_bar, torch.float32, batch.n_struct, "e_bar")
    _want(f_bar, torch.float32, 3 * batch.n_atom, "f_bar")
    _want(v_bar, torch.float32, 6 * batch.n_struct, "v_bar")
    _check(_lib.load().nep_vjp(C.byref(model.c()), C.byref(batch.c()), C.byref(nbrs.c()), _ptr(params),
                               _ptr(e_bar), _ptr(f_bar), _ptr(v_bar), _ptr(grad), _ptr(ws), _stream(stream)),
           "nep_vjp")


class Labels:
    def __init__(self, energy, force, virial):
        self.energy, self.force, self.virial = energy, force, virial

    def c(self):
        return _lib.NepLabels(self.energy.data_ptr(), self.force.data_ptr(), self.virial.data_ptr())


def _lam(lam):
    return (C.c_float * 3)(*[float(x) for x in lam])


def loss_grad(model, batch, nbrs, params, labels: Labels, lam, loss, grad, ws, flags, e_struct=None, force=None,
              virial=None, stream=None):
    P = param_count(model)
    _want(params, torch.float32, P, "params")
    _want(grad, torch.float32, P, "grad")
    _want(loss, torch.float32, 4, "loss")
    _want(labels.energy, torch.float32, batch.n_struct, "labels.energy")
    _want(labels.force, torch.float32, 3 * batch.n_atom, "labels.force")
    _want(labels.virial, torch.float32, 6 * batch.n_struct, "labels.virial")
    _check(_lib.load().nep_loss_grad(C.byref(model.c()), C.byref(batch.c()), C.byref(nbrs.c()), _ptr(params),
                                     C.byref(labels.c()), C.byref(_lam(lam)), _ptr(loss), _ptr(grad),
                                     _ptr(e_struct), _ptr(force), _ptr(virial), _ptr(ws), _ptr(flags),
                                     _stream(stream)), "nep_loss_grad")


STATIC_SCRATCH_BYTES = 64 << 20   # NEP_STATIC_SCRATCH_BYTES


def loss_grad_noalloc(model, batch, nbrs, params, labels: Labels, lam, loss, grad, flags, e_struct=None, force=None,
                      virial=None, stream=None):
    """Neighbor build plus loss and gradient with the library's static device
    scratch in place of a workspace (nep_loss_grad_noalloc); nothing is
    allocated.  Calls on one GPU share the scratch and must not overlap."""
    P = param_count(model)
    _want(params, torch.float32, P, "params")
    _want(grad, torch.float32, P, "grad")
    _want(loss, torch.float32, 4, "loss")
    _want(flags, torch.int32, 1, "flags")
    _want(labels.energy, torch.float32, batch.n_struct, "labels.energy")
    _want(labels.force, torch.float32, 3 * batch.n_atom, "labels.force")
    _want(labels.virial, torch.float32, 6 * batch.n_struct, "labels.virial")
    _check(_lib.load().nep_loss_grad_noalloc(C.byref(model.c()), C.byref(batch.c()), C.byref(nbrs.c()),
                                             _ptr(params), C.byref(labels.c()), C.byref(_lam(lam)), _ptr(loss),
                                             _ptr(grad), _ptr(e_struct), _ptr(force), _ptr(virial), _ptr(flags),
                                             _stream(stream)), "nep_loss_grad_noalloc")


def adam_step(params, m, v, grad, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    P = params.numel()
    for t, name in ((m, "m"), (v, "v"), (grad, "grad")):
        _want(t, torch.float32, P, name)
    _check(_lib.load().nep_adam_step(P, _ptr(params), _ptr(m), _ptr(v), _ptr(grad), lr, beta1, beta2, eps, step,
                                     _stream(stream)), "nep_adam_step")


def lr_schedule(s, lr_start, lr_stop, n_warmup, n_total) -> float:
    return float(_lib.load().nep_lr_schedule(s, lr_start, lr_stop, n_warmup, n_total))


def flags_status(flags_value: int) -> int:
    return int(_lib.load().nep_flags_status(int(flags_value)))


def check_flags(flags, where="device"):
    """Raise NEPError when the device flag word (synchronises) is set."""
    code = flags_status(int(flags.item()))
    _check(code, where)


def md_step(model, batch, nbrs, params, mass, vel, force, dt, n_steps, e_pot, ws, flags, e_kin=None, stream=None):
    """n_steps of velocity Verlet (nep_md_step); batch.pos, vel and force are
    advanced in place, e_pot/e_kin receive per-structure energies."""
    _want(mass, torch.float32, model.n_types, "mass")
    for t, name in ((vel, "vel"), (force, "force")):
        _want(t, torch.float32, 3 * batch.n_atom, name)
    _want(e_pot, torch.float32, batch.n_struct, "e_pot")
    _check(_lib.load().nep_md_step(C.byref(model.c()), C.byref(batch.c()), _ptr(batch.pos), C.byref(nbrs.c()),
                                   _ptr(params), _ptr(mass), _ptr(vel), _ptr(force), float(dt), int(n_steps),
                                   _ptr(e_pot), _ptr(e_kin), _ptr(ws), _ptr(flags), _stream(stream)), "nep_md_step")


TUNING_FIELDS = ("persistent", "outer_blocks_w", "outer_blocks_c", "reduce_chunks", "cell_min_atoms",
                 "gather_lanes", "forward_waves", "adjoint_waves", "reverse_branch")


def tuning_struct(tuning):
    """nep_tuning from a dict of launch choices (missing keys: defaults)."""
    tuning = tuning or {}
    unknown = set(tuning) - set(TUNING_FIELDS)
    if unknown:
        raise ValueError(f"unknown tuning keys {sorted(unknown)}")
    return _lib.NepTuning(*[int(tuning.get(k, 0)) for k in TUNING_FIELDS])


GRAPH_CACHED_NEIGHBORS = 1
GRAPH_PERSISTENT = 2
NEP_FLAG_BARRIER = 64


class TrainStepGraph:
    """One captured training step (neighbors, forward, loss, adjoint, Adam);
    replays advance the device step counter.  With cached_neighbors the graph
    skips the neighbor build and reuses the lists (and the reverse index and
    species order in ws) from an earlier build_neighbors call.  With
    persistent everything after the neighbor build runs as one persistent
    launch (NEP_GRAPH_PERSISTENT).  tuning: launch choices (nep_tuning) as a
    dict, None for the defaults, or "cache" for the autotuner's choice for
    this model and batch size class (defaults when it has none)."""

    def __init__(self, model, batch, nbrs, labels, lam, params, m, v, grad, loss, step, ws, flags,
                 lr_start=1e-3, lr_stop=1e-3, n_warmup=0, n_total=0, beta1=0.9, beta2=0.999, eps=1e-8,
                 stream=None, cached_neighbors=False, persistent=False, tuning="cache"):
        P = param_count(model)
        for t, name in ((params, "params"), (m, "m"), (v, "v"), (grad, "grad")):
            _want(t, torch.float32, P, name)
        _want(step, torch.int32, 1, "step")
        self._keep = (model, batch, nbrs, labels, params, m, v, grad, loss, step, ws, flags)
        cfg = _lib.NepAdamConfig(lr_start, lr_stop, n_warmup, n_total, beta1, beta2, eps)
        if isinstance(tuning, str):
            if tuning != "cache":
                raise ValueError("tuning: a dict of launch choices, None (defaults) or 'cache'")
            from . import tune
            tuning = tune.lookup(model, batch)
        self.tuning = dict(tuning or {})
        if persistent:
            self.tuning["persistent"] = 1
        h = C.c_void_p()
        _check(_lib.load().nep_train_step_graph_create_tuned(
            C.byref(model.c()), C.byref(batch.c()), C.byref(nbrs.c()), C.byref(labels.c()), C.byref(_lam(lam)),
            _ptr(params), _ptr(m), _ptr(v), _ptr(grad), _ptr(loss), _ptr(step), C.byref(cfg), _ptr(ws),
            _ptr(flags), GRAPH_CACHED_NEIGHBORS if cached_neighbors else 0, C.byref(tuning_struct(self.tuning)),
            _stream(stream), C.byref(h)),
            "nep_train_step_graph_create_tuned")
        self.handle = h

    def launch(self, stream=None):
        _check(_lib.load().nep_train_step_graph_launch(self.handle, _stream(stream)), "nep_train_step_graph_launch")

    def close(self):
        if self.handle:
            _lib.load().nep_train_step_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_loss_grad(model, batch, nbrs, params, labels, lam, loss, grad, ws, flags, stream=None, max_kernels=64):
    ms = (C.c_float * max_kernels)()
    names = (C.c_char_p * max_kernels)()
    n = C.c_int32(0)
    _check(_lib.load().nep_profile_loss_grad(C.byref(model.c()), C.byref(batch.c()), C.byref(nbrs.c()),
                                             _ptr(params), C.byref(labels.c()), C.byref(_lam(lam)), _ptr(loss),
                                             _ptr(grad), _ptr(ws), _ptr(flags), _stream(stream), ms, names,
                                             max_kernels, C.byref(n)), "nep_profile_loss_grad")
    return [(names[k].decode(), float(ms[k])) for k in range(min(n.value, max_kernels))]
