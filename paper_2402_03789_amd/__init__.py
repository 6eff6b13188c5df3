"""MI355X-native SevenNet/NequIP energy, force and virial evaluation.

Python layer over libsn.so (include/sn.h): argument marshalling, a
torch.autograd.Function wrapper, and the serving loop.  All arithmetic of
the evaluation runs in the library's gfx950 kernels; nothing here falls back
to a CPU or PyTorch implementation.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref

import numpy as np
import torch

from ._lib import (lib, check, ptr, PRECISIONS, SNError, ModelInfo, EXPORTED,  # noqa: F401
                   Allocator, Batch, ALLOC_FN, FREE_FN)

# contexts still open at interpreter exit are closed while torch (whose allocator may hold
# their memory) is still usable
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for c in list(_LIVE):
        try:
            c.close()
        except Exception:
            pass


def _torch_allocator():
    """sn_allocator_t over torch's caching allocator (memory shows in torch's statistics
    and is reused by torch once the context frees it)."""
    def _alloc(_user, nbytes, device, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, int(stream or 0))
        except Exception:  # out of memory: the library reports SN_ENOMEM
            return None

    def _free(_user, p, _nbytes, _device, _stream):
        torch.cuda.caching_allocator_delete(int(p))

    fa, ff = ALLOC_FN(_alloc), FREE_FN(_free)
    return Allocator(fa, ff, None), (fa, ff)


def cg_table(l1: int, l2: int, l3: int) -> np.ndarray:
    """The library's real Clebsch-Gordan tensor for (l1, l2) -> l3."""
    out = np.zeros((2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1))
    check(lib().sn_cg_table(l1, l2, l3, ptr(out)))
    return out.reshape(2 * l1 + 1, 2 * l2 + 1, 2 * l3 + 1)


class Model:
    """A weights file loaded into host memory (shared by contexts)."""

    def __init__(self, path: str):
        h = C.c_void_p()
        check(lib().sn_model_load(path.encode(), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        i = ModelInfo()
        check(lib().sn_model_info(self._h, C.byref(i)))
        return dict(n_layers=i.n_layers, l_max=i.l_max, l_sh=i.l_sh, muls=list(i.muls)[:i.l_max + 1],
                    n_basis=i.n_basis, hidden=i.hidden, n_species=i.n_species,
                    species=list(i.species_z[:i.n_species]), r_cut=i.r_cut, k_avg=i.k_avg,
                    sigma=i.sigma, n_params=i.n_params)

    def tensors(self) -> list:
        """[(name, offset, count)] of every weight tensor (offsets in float64 values; the
        layout of the weights file and of the training weight gradients)."""
        out = []
        i = 0
        while True:
            name, off, cnt = C.c_char_p(), C.c_int64(), C.c_int64()
            if lib().sn_model_tensor(self._h, i, C.byref(name), C.byref(off), C.byref(cnt)) != 0:
                return out
            out.append((name.value.decode(), off.value, cnt.value))
            i += 1

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().sn_model_free(self._h)
                self._h = None
        except Exception:
            pass


def _device_f64(t, shape):
    """The MD entry points take raw device pointers: refuse anything but a contiguous
    float64 tensor of the expected shape on a GPU."""
    if (not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda
            or not t.is_contiguous() or tuple(t.shape) != tuple(shape)):
        raise ValueError(f"expected a contiguous float64 CUDA tensor of shape {tuple(shape)}")


class Context:
    """One model on one device, stream and precision form."""

    def __init__(self, model: Model, device: int = 0, precision: str = "fp32", skin: float = 0.0,
                 stream=None, hbm_budget: int = 0, allocator: str | None = "torch"):
        """allocator: "torch" serves the context's device memory from torch's caching
        allocator; None lets the library call hipMalloc."""
        self.model = model
        self.device = device
        self.skin = float(skin)  # neighbour-list skin (angstrom) of graph reuse
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self._alloc = None
        alloc_ref = None
        if allocator == "torch":
            self._alloc, self._alloc_keep = _torch_allocator()  # kept alive with the context
            alloc_ref = C.byref(self._alloc)
        elif allocator is not None:
            raise ValueError(f"unknown allocator {allocator!r}")
        self._ones = None
        h = C.c_void_p()
        st = lib().sn_ctx_create(model.handle, device, C.c_void_p(stream.cuda_stream), hbm_budget,
                                 PRECISIONS[precision], float(skin), alloc_ref, C.byref(h))
        check(st)
        self._h = h
        _LIVE.add(self)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().sn_ctx_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def compute(self, pos, Z, cell, forces=True, virial=True, noalloc=False) -> dict:
        """Host-buffer evaluation: E, per-atom E, F, W (float64).  noalloc=True runs
        sn_compute_noalloc (no device allocation: the library's static scratch)."""
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        Z = np.ascontiguousarray(Z, dtype=np.int32)
        cell = np.ascontiguousarray(cell, dtype=np.float64)
        n = pos.shape[0]
        e = np.zeros(1)
        ae = np.zeros(n)
        f = np.zeros((n, 3)) if forces else None
        w = np.zeros((3, 3)) if virial else None
        pbc = (C.c_uint8 * 3)(1, 1, 1)
        fn = lib().sn_compute_noalloc if noalloc else lib().sn_compute
        check(fn(self._h, n, ptr(pos), ptr(Z), ptr(cell), C.cast(pbc, C.c_void_p),
                 ptr(e), ptr(ae), ptr(f), ptr(w)), self._h)
        out = dict(energy=float(e[0]), atom_energy=ae)
        if forces:
            out["forces"] = f
        if virial:
            out["virial"] = w
        return out

    def compute_batch(self, structures, forces=True, virial=True) -> list:
        """Several structures (each (pos, Z, cell)) as one packed graph; per-structure results."""
        B = len(structures)
        offsets = np.zeros(B + 1, dtype=np.int64)
        for b, (p, z, c) in enumerate(structures):
            offsets[b + 1] = offsets[b] + len(z)
        n = int(offsets[-1])
        pos = np.ascontiguousarray(np.concatenate([np.asarray(p, np.float64) for p, _, _ in structures]))
        Z = np.ascontiguousarray(np.concatenate([np.asarray(z, np.int32) for _, z, _ in structures]))
        cells = np.ascontiguousarray(np.stack([np.asarray(c, np.float64) for _, _, c in structures]))
        e = np.zeros(B)
        ae = np.zeros(n)
        f = np.zeros((n, 3)) if forces else None
        w = np.zeros((B, 3, 3)) if virial else None
        check(lib().sn_compute_batch(self._h, B, ptr(offsets), ptr(pos), ptr(Z), ptr(cells), ptr(e),
                                     ptr(ae), ptr(f), ptr(w)), self._h)
        out = []
        for b in range(B):
            a, z = offsets[b], offsets[b + 1]
            r = dict(energy=float(e[b]), atom_energy=ae[a:z])
            if forces:
                r["forces"] = f[a:z]
            if virial:
                r["virial"] = w[b]
            out.append(r)
        return out

    def forward_device(self, pos: torch.Tensor, Z: torch.Tensor, cell, energy: torch.Tensor,
                       atom_energy: torch.Tensor | None = None, offsets=None):
        """Energies of a packed batch in device memory.  pos [n,3] float64 and Z [n] int32 on
        the context's device; offsets (B+1, host) delimit the structures (None: one structure
        of all n atoms); cell: 3x3 or B x 3 x 3 (host).  energy [B] and atom_energy [n]
        (optional) are float64 device outputs."""
        n = int(pos.shape[0])
        offs = np.array([0, n] if offsets is None else offsets, dtype=np.int64)
        B = len(offs) - 1
        cells = np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(B, 9))
        for t, dt in ((pos, torch.float64), (Z, torch.int32), (energy, torch.float64)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"expected a contiguous {dt} device tensor")
        if energy.numel() < B or (atom_energy is not None and atom_energy.numel() < n):
            raise ValueError("output tensor too small")
        b = Batch(B, offs.ctypes.data, cells.ctypes.data, pos.data_ptr(), Z.data_ptr())
        check(lib().sn_forward_device(self._h, C.byref(b), ptr(energy), ptr(atom_energy)), self._h)
        self._pending_B = B

    def backward_device(self, grad_energy, forces: torch.Tensor, virial: torch.Tensor | None):
        """Consume the pending forward.  grad_energy: dL/dE_b as a float64 device tensor [B],
        or a float (every structure).  forces [n,3] <- g_b F_i; virial [B,9] <- g_b W_b."""
        B = getattr(self, "_pending_B", 1)
        if not isinstance(grad_energy, torch.Tensor):
            g = float(grad_energy)
            if g == 1.0:  # kept on the device: MD loops and graph replays reuse it
                if self._ones is None or self._ones.numel() < B:
                    self._ones = torch.ones(max(B, 64), dtype=torch.float64, device=forces.device)
                grad_energy = self._ones
            else:
                grad_energy = torch.full((B,), g, dtype=torch.float64, device=forces.device)
        if grad_energy.dtype != torch.float64 or not grad_energy.is_cuda or grad_energy.numel() < B:
            raise ValueError(f"grad_energy must be a float64 device tensor of at least {B} values")
        grad_energy = grad_energy.contiguous()
        self._g_keep = grad_energy  # alive until the queued backward has read it
        check(lib().sn_backward_device(self._h, ptr(grad_energy), ptr(forces), ptr(virial)), self._h)

    def synchronize(self):
        check(lib().sn_ctx_synchronize(self._h), self._h)

    def set_training(self, on: bool):
        """Later forwards keep what the weight gradients need (sn_ctx_set_training)."""
        check(lib().sn_ctx_set_training(self._h, 1 if on else 0), self._h)

    def backward_train_device(self, grad_energy: torch.Tensor, weight_grad: torch.Tensor,
                              forces: torch.Tensor | None = None, virial: torch.Tensor | None = None):
        """Consume a training-mode forward: weight_grad (float64 device, n_params) <- sum_b g_b
        dE_b/dW with g = grad_energy [B] (float64 device); forces and virial as
        backward_device."""
        for t in (grad_energy, weight_grad):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("expected contiguous float64 device tensors")
        if weight_grad.numel() < self.model.info()["n_params"]:
            raise ValueError("weight_grad too small")
        check(lib().sn_backward_train_device(self._h, ptr(grad_energy), ptr(forces), ptr(virial),
                                             ptr(weight_grad)), self._h)

    def graph_size(self):
        n, g, e = C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().sn_ctx_graph_size(self._h, C.byref(n), C.byref(g), C.byref(e)))
        return n.value, g.value, e.value

    def set_domains(self, nx: int, ny: int = 1, nz: int = 1):
        """Evaluate later calls as nx x ny x nz subdomains, each with its own ghost shell."""
        check(lib().sn_ctx_set_domains(self._h, int(nx), int(ny), int(nz)), self._h)

    def set_capture(self, on: bool):
        """Replay reused-neighbour-list evaluations from a recorded HIP graph."""
        check(lib().sn_ctx_set_capture(self._h, 1 if on else 0), self._h)

    def set_edge_compaction(self, on: bool):
        """Evaluate lists built with a skin over their pairs inside r_c only (default on);
        takes effect at the next list build."""
        check(lib().sn_ctx_set_edge_compaction(self._h, 1 if on else 0))

    def evaluated_edges(self):
        """(directed edges, pairs) the last forward evaluated."""
        e, p = C.c_int64(), C.c_int64()
        check(lib().sn_ctx_evaluated_edges(self._h, C.byref(e), C.byref(p)))
        return e.value, p.value

    def set_graph_reuse(self, reuse: bool):
        check(lib().sn_ctx_set_graph_reuse(self._h, 1 if reuse else 0))

    def verlet(self, pos, vel, forces, inv_mass, dt: float, stage: int):
        n = pos.shape[0]
        for t, shape in ((pos, (n, 3)), (vel, (n, 3)), (forces, (n, 3)), (inv_mass, (n,))):
            _device_f64(t, shape)
        check(lib().sn_md_verlet(self._h, n, ptr(pos), ptr(vel), ptr(forces),
                                 ptr(inv_mass), float(dt), int(stage)), self._h)

    def nh_half(self, vel, inv_mass, dt: float, kT: float, dof: float, Q: float, state):
        """Thermostat half NH(dt/2) of a Nose-Hoover step of length dt on device velocities;
        state: 4 float64 on the device ({xi, eta, scale, K}, zeros before the first call)."""
        n = vel.shape[0]
        for t, shape in ((vel, (n, 3)), (inv_mass, (n,)), (state, (4,))):
            _device_f64(t, shape)
        check(lib().sn_md_nh_half(self._h, n, ptr(vel), ptr(inv_mass), float(dt), float(kT),
                                  float(dof), float(Q), ptr(state)), self._h)

    def max_displacement(self, pos, ref) -> float:
        """max_i |pos_i - ref_i| (angstrom) of two n x 3 float64 device arrays."""
        n = pos.shape[0]
        for t in (pos, ref):
            _device_f64(t, (n, 3))
        v = C.c_double()
        check(lib().sn_md_max_displacement(self._h, n, ptr(pos), ptr(ref), C.byref(v)), self._h)
        return v.value

    def memory(self) -> int:
        v = C.c_size_t()
        check(lib().sn_ctx_memory(self._h, C.byref(v)))
        return v.value

    def n_pairs(self) -> int:
        v = C.c_int64()
        check(lib().sn_ctx_pair_count(self._h, C.byref(v)))
        return v.value

    def graph(self) -> dict:
        n, g, e = self.graph_size()
        recv = np.zeros(e, np.int32)
        send = np.zeros(e, np.int32)
        shift = np.zeros((e, 3), np.int32)
        gown = np.zeros(g, np.int32)
        gsh = np.zeros((g, 3), np.int32)
        check(lib().sn_ctx_graph(self._h, ptr(recv), ptr(send), ptr(shift), ptr(gown), ptr(gsh)),
              self._h)
        return dict(recv=recv, send_owner=send, shift=shift, ghost_owner=gown, ghost_shift=gsh)

    def timings(self) -> dict:
        cnt = C.c_int(256)
        names = (C.c_char_p * 256)()
        ms = np.zeros(256)
        check(lib().sn_ctx_timings(self._h, names, ptr(ms), C.byref(cnt)))
        return {names[i].decode(): float(ms[i]) for i in range(min(cnt.value, 256))}


class SevenNetEnergy(torch.autograd.Function):
    """Energies of a packed batch with forces from the library's hand-written adjoint.

    forward(pos [n,3] float64 cuda, Z [n] int32 cuda, cells (B x 3 x 3 host), offsets (B+1 host
    int64, or None for one structure), ctx) -> E [B] float64; backward takes dL/dE [B] on the
    device (no host synchronisation) and gives dL/dpos = -g_b F_i.  The virials of the last
    backward (g_b W_b, [B,9]) are stored on the context object as `last_virial`.
    """

    @staticmethod
    def forward(actx, pos, Z, cells, offsets, ctx: Context):
        n = int(pos.shape[0])
        offs = np.array([0, n] if offsets is None else offsets, dtype=np.int64)
        B = len(offs) - 1
        energy = torch.zeros(B, dtype=torch.float64, device=pos.device)
        ctx.forward_device(pos.contiguous(), Z.contiguous(), cells, energy, offsets=offs)
        actx.sn = ctx
        actx.n = n
        actx.B = B
        return energy

    @staticmethod
    def backward(actx, grad_e):
        ctx = actx.sn
        g = grad_e.to(torch.float64).contiguous()
        f = torch.empty((actx.n, 3), dtype=torch.float64, device=grad_e.device)
        w = torch.empty((actx.B, 9), dtype=torch.float64, device=grad_e.device)
        ctx.backward_device(g, f, w)
        ctx.last_virial = w
        return -f, None, None, None, None


def energy(pos, Z, cell, ctx: Context):
    """Total energy of one structure (scalar) through SevenNetEnergy."""
    return SevenNetEnergy.apply(pos, Z, cell, None, ctx)[0]


def energies(pos, Z, cells, offsets, ctx: Context):
    """Energies [B] of a packed batch through SevenNetEnergy."""
    return SevenNetEnergy.apply(pos, Z, cells, offsets, ctx)
