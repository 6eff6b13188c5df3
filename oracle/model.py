"""The NequIP-architecture model of SevenNet, evaluated in float64 on CPU.

TEST INFRASTRUCTURE (see oracle/__init__.py).

Model (paper section 2.2 and section 5.1; where the paper leaves a point open,
the reading taken is the one written here):

  h^(1)_i = W_emb[s_i]                               (scalars only)
  for each interaction block t:
    x   = Lin1(h)          per-degree channel mixing
    sc  = Linsc(h)         linear self-connection (replaces the species TP)
    w_e = phi(phi(rho_e Wa) Wb) Wc                  radial MLP, no biases
    q_e,p[u, m3] = w_e[p, u] sum_{m1, m2} C^p[m1, m2, m3] x_src[l1][u, m1] Y^{l2}_e[m2]
    M_i = (1 / k_avg) sum_{e: recv(e) = i} q_e      (channels of the paths with
                                                     the same l3, in path order)
    y   = Lin2(M) + sc
    h'  = gate(y): phi on the first C0 scalars; each l > 0 channel times
          phi(its gate scalar); the last block keeps only scalar paths and
          applies phi to all its outputs
  E_i = sigma (h_i Wr1) Wr2 + mu_{s_i},   E = sum_i E_i          (eq 1)
  phi(z) = c z sigmoid(z), c = 1 / sqrt(E[SiLU(z)^2]), z ~ N(0, 1)

Forces follow eq 2 through autograd, and are also assembled from the edge
gradients g_e = dE/dd_e as in eqs 5-6:
  F_k = sum_{e: recv=k} g_e - sum_{e: owner(send)=k} g_e
The virial is W = -sum_e d_e (x) g_e (eV).
"""
from __future__ import annotations

import math

import numpy as np
import torch
from torch.utils.checkpoint import checkpoint

from .basis import real_sph_harm, radial_basis
from .cg import real_cg
from .graph import periodic_edges, wrap, ghost_shell, subdomains

DT = torch.float64


class OracleModel:
    """Holds the configuration, weights and per-block path lists."""

    def __init__(self, config: dict, weights: dict):
        self.cfg = dict(config)
        self.T = int(config["n_layers"])
        self.muls = [int(m) for m in config["muls"]]
        self.lmax = len(self.muls) - 1
        self.lsh = int(config["l_sh"])
        self.rc = float(config["r_cut"])
        self.nb = int(config["n_basis"])
        self.p = int(config["envelope_p"])
        self.kavg = float(config["k_avg"])
        self.sigma = float(config["sigma"])
        self.species = [int(z) for z in config["species"]]
        self.shift = torch.tensor([float(v) for v in config["shift"]], dtype=DT)
        self.c = float(config["act_scale"])
        if config.get("gate", "silu") != "silu":
            raise ValueError("only SiLU gates are defined")
        self.C0 = self.muls[0]
        # receivers are processed in chunks of about this many edges when a structure has
        # more (memory bound of the autograd graph; the result does not depend on it)
        self.chunk_edges = 200_000
        self.W = {k: torch.as_tensor(np.asarray(v), dtype=DT) for k, v in weights.items()}
        self.layers = []
        for t in range(self.T):
            last = t == self.T - 1
            ins = [0] if t == 0 else [l for l in range(self.lmax + 1) if self.muls[l] > 0]
            outs = [0] if last else [l for l in range(self.lmax + 1) if self.muls[l] > 0]
            paths = [(l1, l2, l3) for l1 in ins for l2 in range(self.lsh + 1)
                     for l3 in range(abs(l1 - l2), min(l1 + l2, self.lmax) + 1) if l3 in outs]
            if last:
                gmul = {0: self.C0}
            else:
                gmul = {l: (sum(self.muls) if l == 0 else self.muls[l]) for l in outs}
            self.layers.append(dict(last=last, ins=ins, outs=outs, paths=paths, gmul=gmul))
        self.cg = {p: torch.as_tensor(real_cg(*p), dtype=DT)
                   for L in self.layers for p in L["paths"]}
        self._check_shapes()

    def _check_shapes(self):
        W = self.W
        assert tuple(W["embed"].shape) == (len(self.species), self.C0)
        for t, L in enumerate(self.layers):
            for l in L["ins"]:
                assert tuple(W[f"l{t}.lin1.{l}"].shape) == (self.muls[l], self.muls[l])
                if l in L["gmul"]:
                    assert tuple(W[f"l{t}.linsc.{l}"].shape) == (self.muls[l], L["gmul"][l])
            P = sum(self.muls[l1] for (l1, _, _) in L["paths"])
            assert W[f"l{t}.mlp.2"].shape[1] == P
            for l in L["outs"]:
                mid = sum(self.muls[l1] for (l1, _, l3) in L["paths"] if l3 == l)
                assert tuple(W[f"l{t}.lin2.{l}"].shape) == (mid, L["gmul"][l])

    def n_params(self) -> int:
        return int(sum(v.numel() for v in self.W.values()))

    def species_index(self, Z) -> torch.Tensor:
        lut = {z: i for i, z in enumerate(self.species)}
        return torch.tensor([lut[int(z)] for z in Z], dtype=torch.long)

    # ---- pieces of one interaction block -------------------------------------------
    def phi(self, z):
        return self.c * z * torch.sigmoid(z)

    @staticmethod
    def lin(h: torch.Tensor, Wm: torch.Tensor) -> torch.Tensor:
        # h [n, u, m], W [u, v] -> [n, v, m]
        return torch.einsum("num,uv->nvm", h, Wm)

    def radial_weights(self, t: int, rho: torch.Tensor) -> torch.Tensor:
        W = self.W
        a = self.phi(rho @ W[f"l{t}.mlp.0"])
        a = self.phi(a @ W[f"l{t}.mlp.1"])
        return a @ W[f"l{t}.mlp.2"]

    def _conv_chunk(self, t, n_recv, recv, send, Y, rho, *xs):
        """Messages of one receiver range: returns per-l3 tensors [n_recv, mid, 2l3+1]."""
        L = self.layers[t]
        x = dict(zip(L["ins"], xs))
        w = self.radial_weights(t, rho)
        parts = {l: [] for l in L["outs"]}
        off = 0
        for (l1, l2, l3) in L["paths"]:
            mul = self.muls[l1]
            xs_e = x[l1][send]                                   # [E, u, 2l1+1]
            tp = torch.einsum("eui,ej,ijk->euk", xs_e, Y[l2], self.cg[(l1, l2, l3)])
            q = w[:, off:off + mul, None] * tp
            m = torch.zeros(n_recv, mul, 2 * l3 + 1, dtype=DT).index_add_(0, recv, q)
            parts[l3].append(m)
            off += mul
        return tuple(torch.cat(parts[l], dim=1) / self.kavg for l in L["outs"])

    def conv(self, t, x_send: dict, recv, send, n_recv, Y, rho, chunk_edges=None):
        """Aggregated messages M[l3] for receivers 0..n_recv-1 (edges sorted by receiver)."""
        L = self.layers[t]
        if chunk_edges is None:
            chunk_edges = self.chunk_edges
        xs = [x_send[l] for l in L["ins"]]
        E = recv.shape[0]
        if E <= chunk_edges:
            return dict(zip(L["outs"], self._conv_chunk(t, n_recv, recv, send, Y, rho, *xs)))
        # receiver-aligned chunks, each recomputed in the backward pass
        bounds = torch.searchsorted(recv, torch.arange(0, n_recv + 1, dtype=recv.dtype))
        outs = {l: [] for l in L["outs"]}
        r0 = 0
        while r0 < n_recv:
            e0 = int(bounds[r0])
            r1 = int(torch.searchsorted(bounds, torch.tensor(e0 + chunk_edges), right=True)) - 1
            r1 = max(r1, r0 + 1)
            r1 = min(r1, n_recv)
            e1 = int(bounds[r1])
            res = checkpoint(self._conv_chunk, t, r1 - r0, recv[e0:e1] - r0, send[e0:e1],
                             [y[e0:e1] for y in Y], rho[e0:e1], *xs, use_reentrant=False)
            for l, m in zip(L["outs"], res):
                outs[l].append(m)
            r0 = r1
        return {l: torch.cat(v, dim=0) for l, v in outs.items()}

    def gate(self, t, y: dict) -> dict:
        L = self.layers[t]
        if L["last"]:
            return {0: self.phi(y[0])}
        C0 = self.C0
        h = {0: self.phi(y[0][:, :C0])}
        g = self.phi(y[0][:, C0:, 0])
        off = 0
        for l in L["outs"]:
            if l == 0:
                continue
            h[l] = g[:, off:off + self.muls[l], None] * y[l]
            off += self.muls[l]
        return h

    def readout(self, h0: torch.Tensor, s_idx: torch.Tensor) -> torch.Tensor:
        W = self.W
        eps = (h0[:, :, 0] @ W["readout.0"]) @ W["readout.1"]
        return self.sigma * eps[:, 0] + self.shift[s_idx]

    def edge_features(self, d: torch.Tensor):
        r = torch.linalg.norm(d, dim=1)
        Y = real_sph_harm(d / r[:, None], self.lsh)
        rho = radial_basis(r, self.rc, self.nb, self.p)
        return Y, rho

    def embed(self, s_idx: torch.Tensor) -> dict:
        return {0: self.W["embed"][s_idx][:, :, None]}


# ---- whole-box periodic evaluation (the definition) ------------------------------------

def _finish(model, E_i, ds, pos_t, recv, owner_of_send, n_atoms):
    E = E_i.sum()
    grads = torch.autograd.grad(E, list(ds) + [pos_t], allow_unused=True)
    g = torch.cat([gi if gi is not None else torch.zeros_like(di)
                   for gi, di in zip(grads[:-1], ds)])
    gpos = grads[-1]
    d = torch.cat(list(ds))
    F = torch.zeros(n_atoms, 3, dtype=DT)
    F.index_add_(0, recv, g)
    F.index_add_(0, owner_of_send, -g)
    W = -(d.detach().T @ g)
    return dict(energy=float(E), atom_energy=E_i.detach().numpy(), forces=F.numpy(),
                forces_autograd=(-gpos).numpy(), virial=W.numpy(), edge_grad=g.numpy(),
                d=d.detach().numpy())


def atom_energies(model: OracleModel, pos, Z, cell, pbc=(True, True, True), graph=None):
    """Per-atom energies E_i (paper eq 1) of one periodic structure as a tensor that carries
    the autograd graph back to the positions and the model's weight tensors.  Returns
    (E_i, edge vectors d, positions tensor, graph)."""
    cell = np.asarray(cell, dtype=np.float64)
    posw = wrap(np.asarray(pos, dtype=np.float64), cell, pbc)
    if graph is None:
        graph = periodic_edges(posw, cell, model.rc, pbc)
    recv, send, shift = (torch.as_tensor(a) for a in graph)
    N = posw.shape[0]
    pos_t = torch.tensor(posw, dtype=DT, requires_grad=True)
    cell_t = torch.tensor(cell, dtype=DT)
    d = pos_t[send] + shift.to(DT) @ cell_t - pos_t[recv]
    Y, rho = model.edge_features(d)
    s_idx = model.species_index(Z)
    h = model.embed(s_idx)
    W = model.W
    for t, L in enumerate(model.layers):
        x = {l: model.lin(h[l], W[f"l{t}.lin1.{l}"]) for l in L["ins"]}
        sc = {l: model.lin(h[l], W[f"l{t}.linsc.{l}"]) for l in L["ins"] if l in L["gmul"]}
        M = model.conv(t, x, recv, send, N, Y, rho)
        y = {}
        for l in L["outs"]:
            y[l] = model.lin(M[l], W[f"l{t}.lin2.{l}"])
            if l in sc:
                y[l] = y[l] + sc[l]
        h = model.gate(t, y)
    return model.readout(h[0], s_idx), d, pos_t, graph


def evaluate(model: OracleModel, pos, Z, cell, pbc=(True, True, True), graph=None):
    """E, per-atom E, F (eq 6 assembly), F (autograd), W for one periodic structure."""
    E_i, d, pos_t, graph = atom_energies(model, pos, Z, cell, pbc, graph)
    recv, send = (torch.as_tensor(a) for a in graph[:2])
    out = _finish(model, E_i, [d], pos_t, recv, send, pos_t.shape[0])
    out["graph"] = (graph[0], graph[1], graph[2])
    return out


# ---- subdomains with ghost shells (the paper's scheme, section 3.1) ------------------

def evaluate_domains(model: OracleModel, pos, Z, cell, domains, pbc=(True, True, True)):
    """Evaluate with the atoms split over subdomains that exchange ghost data.

    Each domain dict has global `local` ids, `ghost_owner` (global ids),
    `ghost_shift`, and edges (`recv` local row, `send` row of [locals, ghosts]).
    Per block t >= 2 every domain's ghost features are refreshed from the
    owners' rows (forward communication); in block 1 a ghost's features come
    from its own species, so no refresh is needed.  Autograd carries the
    reverse communication: gradients reaching ghost rows and ghost positions
    flow back to the owners.
    """
    cell = np.asarray(cell, dtype=np.float64)
    posw = wrap(np.asarray(pos, dtype=np.float64), cell, pbc)
    N = posw.shape[0]
    pos_t = torch.tensor(posw, dtype=DT, requires_grad=True)
    cell_t = torch.tensor(cell, dtype=DT)
    s_all = model.species_index(Z)
    W = model.W
    dom = []
    for D in domains:
        loc = torch.as_tensor(D["local"])
        own = torch.as_tensor(D["ghost_owner"])
        shf = torch.as_tensor(D["ghost_shift"]).to(DT)
        recv = torch.as_tensor(D["recv"])
        send = torch.as_tensor(D["send"])
        # forward communication of positions and species (fig 3c)
        p_ext = torch.cat([pos_t[loc], pos_t[own] + shf @ cell_t])
        d = p_ext[send] - p_ext[recv]
        Y, rho = model.edge_features(d)
        dom.append(dict(loc=loc, own=own, recv=recv, send=send, d=d, Y=Y, rho=rho,
                        s_loc=s_all[loc], s_gh=s_all[own], n=len(loc)))
    h = [model.embed(D["s_loc"]) for D in dom]
    h_gh = [model.embed(D["s_gh"]) for D in dom]
    for t, L in enumerate(model.layers):
        xs = [{l: model.lin(h[k][l], W[f"l{t}.lin1.{l}"]) for l in L["ins"]} for k in range(len(dom))]
        if t == 0:
            # ghost rows from their own species: no communication in block 1
            xg = [{l: model.lin(h_gh[k][l], W[f"l{t}.lin1.{l}"]) for l in L["ins"]}
                  for k in range(len(dom))]
        else:
            # forward communication of node features (fig 3d)
            glob = {}
            for l in L["ins"]:
                buf = torch.zeros(N, *xs[0][l].shape[1:], dtype=DT)
                for k, D in enumerate(dom):
                    buf = buf.index_copy(0, D["loc"], xs[k][l])
                glob[l] = buf
            xg = [{l: glob[l][D["own"]] for l in L["ins"]} for D in dom]
        new_h = []
        for k, D in enumerate(dom):
            x_ext = {l: torch.cat([xs[k][l], xg[k][l]]) for l in L["ins"]}
            sc = {l: model.lin(h[k][l], W[f"l{t}.linsc.{l}"]) for l in L["ins"] if l in L["gmul"]}
            M = model.conv(t, x_ext, D["recv"], D["send"], D["n"], D["Y"], D["rho"])
            y = {}
            for l in L["outs"]:
                y[l] = model.lin(M[l], W[f"l{t}.lin2.{l}"])
                if l in sc:
                    y[l] = y[l] + sc[l]
            new_h.append(model.gate(t, y))
        h = new_h
    E_i = torch.zeros(N, dtype=DT)
    for k, D in enumerate(dom):
        E_i = E_i.index_copy(0, D["loc"], model.readout(h[k][0], D["s_loc"]))
    # global pooling of the energy
    recv_g = torch.cat([D["loc"][D["recv"]] for D in dom])
    send_owner = torch.cat([torch.cat([D["loc"], D["own"]])[D["send"]] for D in dom])
    return _finish(model, E_i, [D["d"] for D in dom], pos_t, recv_g, send_owner, N)


def evaluate_ghost(model: OracleModel, pos, Z, cell, skin=0.0, pbc=(True, True, True)):
    """One subdomain = the whole cell, with a ghost shell of width r_c + skin."""
    cell = np.asarray(cell, dtype=np.float64)
    posw = wrap(np.asarray(pos, dtype=np.float64), cell, pbc)
    D = ghost_shell(posw, cell, model.rc, skin, pbc)
    return evaluate_domains(model, posw, Z, cell, [D], pbc)


def evaluate_subdomains(model: OracleModel, pos, Z, cell, splits=(2, 1, 1), skin=0.0):
    cell = np.asarray(cell, dtype=np.float64)
    posw = wrap(np.asarray(pos, dtype=np.float64), cell)
    doms = subdomains(posw, cell, model.rc, splits, skin)
    return evaluate_domains(model, posw, Z, cell, doms)


def energy_only(model: OracleModel, pos, Z, cell, pbc=(True, True, True)) -> float:
    """Total energy without derivatives (for finite differences)."""
    with torch.enable_grad():
        return evaluate(model, pos, Z, cell, pbc)["energy"]
