"""FP64 reference ("oracle") for one loss-and-gradient evaluation of a NEP
potential over a batch of periodic structures.

TEST INFRASTRUCTURE ONLY.  This is the plain, slow definition that the GPU
library is checked against.  Only tests, the smoke check and the CPU-baseline
leg of the benchmark may import it; the library never does, and nothing here
calls the library.

What it computes, in the paper's order (Sec. II):
  * neighbor sets within r_c (Eq. 2) under periodic boundaries of an
    orthorhombic or triclinic cell, brute force over every atom and every
    image shift in {-1,0,1}^3;
  * radial descriptors q_n (Eqs. 5-6) with the Chebyshev basis and cosine
    cutoff of Appendix A;
  * 3-body angular descriptors q_nl (Eqs. 7-8) from the Cartesian harmonics of
    Appendix B, plus 4-body and 5-body invariants of the same sums;
  * one tanh hidden layer per species giving E_i (Eq. 1, D1.1);
  * forces F = -dE/dr and virials W = -dE/d(strain) (Eqs. 3-4);
  * the weighted loss (Eqs. 9-12) and its exact gradient with respect to
    every parameter (Eqs. 13-16, D1.18-D1.21).
Forces, virials and the parameter gradient are obtained by differentiating
the energy definition with torch autograd in float64: they are the plain
definitions, not the paper's hand-derived chain (the GPU path implements that
chain).  Parity of this module is pinned in tests against closed forms,
central finite differences and invariances.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import harmonics as hm

DT = torch.float64

# image shifts in canonical code order: code = 9(sx+1) + 3(sy+1) + (sz+1)
SHIFTS = np.array([[sx, sy, sz] for sx in (-1, 0, 1) for sy in (-1, 0, 1) for sz in (-1, 0, 1)],
                  dtype=np.float64)
SELF_CODE = 13


@dataclass(frozen=True)
class Sizes:
    """NEP hyper-parameters as counts (n_rad radial channels, k_rad basis
    functions k = 0..k_rad-1, 3-body degrees l = 1..l3, l4 in {0,2},
    l5 in {0,1})."""
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

    @classmethod
    def of(cls, s):
        return cls(s.n_types, s.n_rad, s.n_ang, s.k_rad, s.k_ang, s.l3, s.l4, s.l5,
                   s.hidden, float(s.rc_rad), float(s.rc_ang))

    @property
    def lmax(self) -> int:
        return max(self.l3, self.l4, self.l5)

    @property
    def n_desc(self) -> int:
        return (self.n_rad + self.n_ang * self.l3
                + (self.n_ang if self.l4 else 0) + (self.n_ang if self.l5 else 0))

    @property
    def nn_block(self) -> int:
        return self.hidden * self.n_desc + 2 * self.hidden + 1

    @property
    def n_params(self) -> int:
        t2 = self.n_types ** 2
        return t2 * (self.n_rad * self.k_rad + self.n_ang * self.k_ang) + self.n_types * self.nn_block


def unpack(sz: Sizes, theta: torch.Tensor) -> dict:
    """Parameter vector layout: c^R[I][J][n][k], then c^A[I][J][n][k], then for
    each species I: W0 [hidden][n_desc] (row = hidden unit), b0 [hidden],
    w1 [hidden], b1."""
    T, H, D = sz.n_types, sz.hidden, sz.n_desc
    o = 0
    nr = T * T * sz.n_rad * sz.k_rad
    c_rad = theta[o:o + nr].reshape(T, T, sz.n_rad, sz.k_rad); o += nr
    na = T * T * sz.n_ang * sz.k_ang
    c_ang = theta[o:o + na].reshape(T, T, sz.n_ang, sz.k_ang); o += na
    W0, b0, w1, b1 = [], [], [], []
    for _ in range(T):
        W0.append(theta[o:o + H * D].reshape(H, D)); o += H * D
        b0.append(theta[o:o + H]); o += H
        w1.append(theta[o:o + H]); o += H
        b1.append(theta[o]); o += 1
    assert o == sz.n_params
    return dict(c_rad=c_rad, c_ang=c_ang, W0=torch.stack(W0), b0=torch.stack(b0),
                w1=torch.stack(w1), b1=torch.stack(b1))


# ----------------------------------------------------------------------------
# neighbors (Eq. 2)
# ----------------------------------------------------------------------------
def shift_vectors(box32, tilt32=None) -> np.ndarray:
    """[27, 3] image shifts H s in code order, H the cell matrix with edge
    vectors a = (lx,0,0), b = (xy,ly,0), c = (xz,yz,lz); each component is
    summed in a fixed order: x = ((sa lx) + sb xy) + sc xz, y = sb ly + sc yz,
    z = sc lz (products exact: s is 0 or +-1)."""
    lx, ly, lz = np.asarray(box32, np.float32).astype(np.float64)
    xy, xz, yz = (0.0, 0.0, 0.0) if tilt32 is None else np.asarray(tilt32, np.float32).astype(np.float64)
    sa, sb, sc = SHIFTS[:, 0], SHIFTS[:, 1], SHIFTS[:, 2]
    return np.stack([sa * lx + sb * xy + sc * xz, sb * ly + sc * yz, sc * lz], 1)


def neighbor_pairs(pos32: np.ndarray, box32: np.ndarray, rc: float, rows=None, tilt32=None):
    """All (i, j, code) with |x_j + H s - x_i| < r_c, (j, s) != (i, 0),
    s in {-1,0,1}^3, in canonical order (i, then j, then code ascending).

    The predicate is evaluated in IEEE float64 on the float32 inputs as
    d = (x_j - x_i) + H s, each component summed left to right as
    dx = (((x_j - x_i) + sa lx) + sb xy) + sc xz, dy = ((y_j - y_i) + sb ly) + sc yz,
    dz = (z_j - z_i) + sc lz, and d2 = (dx*dx + dy*dy) + dz*dz, compared with
    r_c^2 strictly.  With zero tilts this is (x_j - x_i) + s L.  `rows`
    restricts the centers i.  Pruning tests, implied by the predicate, only
    skip work."""
    if tilt32 is not None and np.any(np.asarray(tilt32, np.float32) != 0):
        return _neighbor_pairs_triclinic(pos32, box32, rc, rows, tilt32)
    x = np.asarray(pos32, np.float32).astype(np.float64)
    L = np.asarray(box32, np.float32).astype(np.float64)
    rc64 = float(np.float32(rc))
    rc2 = rc64 * rc64
    n = x.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    SL = SHIFTS * L  # exact: shifts are 0 or +-1
    axis_shift = np.array([-1.0, 0.0, 1.0])
    out = []
    chunk = max(1, min(256, 4_000_000 // max(n, 1)))
    for c0 in range(0, len(rows), chunk):
        ii = rows[c0:c0 + chunk]
        diff = x[None, :, :] - x[ii][:, None, :]                        # [c, n, 3]
        near = np.ones(diff.shape[:2], bool)
        for a in range(3):
            da = diff[:, :, a, None] + axis_shift[None, None, :] * L[a]  # [c, n, 3]
            near &= np.any(np.abs(da) < rc64, axis=2)
        ci, cj = np.nonzero(near)
        if len(ci) == 0:
            continue
        d = diff[ci, cj][:, None, :] + SL[None, :, :]                  # [m, 27, 3]
        d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        ok = d2 < rc2
        ok &= ~((ii[ci] == cj)[:, None] & (np.arange(27) == SELF_CODE)[None, :])
        m, code = np.nonzero(ok)
        out.append(np.stack([ii[ci[m]], cj[m], code], 1))
    if not out:
        return np.zeros((0, 3), np.int64)
    p = np.concatenate(out, 0)
    order = np.lexsort((p[:, 2], p[:, 1], p[:, 0]))
    return p[order].astype(np.int64)


def _neighbor_pairs_triclinic(pos32, box32, rc, rows, tilt32):
    x = np.asarray(pos32, np.float32).astype(np.float64)
    lx, ly, lz = np.asarray(box32, np.float32).astype(np.float64)
    xy, xz, yz = np.asarray(tilt32, np.float32).astype(np.float64)
    rc64 = float(np.float32(rc))
    rc2 = rc64 * rc64
    n = x.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    sa, sb, sc = SHIFTS[:, 0], SHIFTS[:, 1], SHIFTS[:, 2]
    out = []
    chunk = max(1, min(256, 2_000_000 // max(n, 1)))
    for c0 in range(0, len(rows), chunk):
        ii = rows[c0:c0 + chunk]
        diff = x[None, :, :] - x[ii][:, None, :]                        # [c, n, 3]
        # |dz| < rc for some sc (dz depends on sc only)
        dzc = diff[:, :, 2, None] + np.array([-lz, 0.0, lz])[None, None, :]
        ci, cj = np.nonzero(np.any(np.abs(dzc) < rc64, axis=2))
        if len(ci) == 0:
            continue
        dd = diff[ci, cj]                                               # [m, 3]
        dx = ((dd[:, 0, None] + sa * lx) + sb * xy) + sc * xz
        dy = (dd[:, 1, None] + sb * ly) + sc * yz
        dz = dd[:, 2, None] + sc * lz
        d2 = (dx * dx + dy * dy) + dz * dz
        ok = d2 < rc2
        ok &= ~((ii[ci] == cj)[:, None] & (np.arange(27) == SELF_CODE)[None, :])
        m, code = np.nonzero(ok)
        out.append(np.stack([ii[ci[m]], cj[m], code], 1))
    if not out:
        return np.zeros((0, 3), np.int64)
    p = np.concatenate(out, 0)
    order = np.lexsort((p[:, 2], p[:, 1], p[:, 0]))
    return p[order].astype(np.int64)


def pair_vectors(pos32: np.ndarray, box32: np.ndarray, pairs: np.ndarray, tilt32=None) -> torch.Tensor:
    """d_ij = x_j + H s - x_i in float64 for each (i, j, code)."""
    x = np.asarray(pos32, np.float32).astype(np.float64)
    i, j, c = pairs[:, 0], pairs[:, 1], pairs[:, 2]
    return torch.tensor((x[j] - x[i]) + shift_vectors(box32, tilt32)[c], dtype=DT)


# ----------------------------------------------------------------------------
# basis (Appendix A)
# ----------------------------------------------------------------------------
def chebyshev(xi: torch.Tensor, K: int) -> torch.Tensor:
    """T_0..T_{K-1} by the three-term recursion (A1.1), stacked last."""
    T = [torch.ones_like(xi)]
    if K > 1:
        T.append(xi)
    for k in range(2, K):
        T.append(2 * xi * T[k - 1] - T[k - 2])
    return torch.stack(T, -1)


def cutoff(r: torch.Tensor, rc: float) -> torch.Tensor:
    """f_c (A2.1)."""
    return torch.where(r <= rc, 0.5 * (1 + torch.cos(math.pi * r / rc)), torch.zeros_like(r))


def radial_functions(r: torch.Tensor, rc: float, K: int) -> torch.Tensor:
    """f_k(r) = (T_k(xi) + 1)/2 * f_c(r), xi = 2(r/r_c - 1)^2 - 1 (Eq. 6, A1.2)."""
    xi = 2 * (r / rc - 1) ** 2 - 1
    return 0.5 * (chebyshev(xi, K) + 1) * cutoff(r, rc)[..., None]


# ----------------------------------------------------------------------------
# descriptors and energy
# ----------------------------------------------------------------------------
class NEPOracle:
    def __init__(self, sizes):
        self.sz = Sizes.of(sizes)
        self.Y = hm.n_harmonics(self.sz.lmax)
        self.clm = torch.tensor(hm.clm_table(self.sz.lmax), dtype=DT)

    # -- descriptor G_i (Eqs. 5-8) ------------------------------------------
    def descriptors(self, p: dict, types: torch.Tensor, n: int,
                    pr: np.ndarray, d_rad: torch.Tensor,
                    pa: np.ndarray, d_ang: torch.Tensor) -> torch.Tensor:
        sz = self.sz
        ti = torch.as_tensor(types, dtype=torch.long)
        # radial: q_n = sum_j g_n(r_ij), g_n = sum_k c_nk^{IJ} f_k
        ir, jr = torch.as_tensor(pr[:, 0]), torch.as_tensor(pr[:, 1])
        r = torch.linalg.norm(d_rad, dim=-1)
        f = radial_functions(r, sz.rc_rad, sz.k_rad)                        # [P, K]
        c = p["c_rad"][ti[ir], ti[jr]]                                       # [P, nR, K]
        g = torch.einsum("pnk,pk->pn", c, f)
        q_rad = torch.zeros(n, sz.n_rad, dtype=DT).index_add(0, ir, g)
        parts = [q_rad]
        if sz.n_ang > 0 and (sz.l3 or sz.l4 or sz.l5):
            ia, ja = torch.as_tensor(pa[:, 0]), torch.as_tensor(pa[:, 1])
            ra = torch.linalg.norm(d_ang, dim=-1)
            fa = radial_functions(ra, sz.rc_ang, sz.k_ang)
            ca = p["c_ang"][ti[ia], ti[ja]]
            ga = torch.einsum("pnk,pk->pn", ca, fa)                          # [P, nA]
            B = hm.B_dir(sz.lmax, d_ang)                                     # [P, Y]
            # S_nlm = sum_j g_n(r_ij) b_lm / r^l  (Eq. 8)
            S = torch.zeros(n, sz.n_ang, self.Y, dtype=DT).index_add(0, ia, ga[:, :, None] * B[:, None, :])
            for l in range(1, sz.l3 + 1):
                a, b = hm.harmonic_index(l, 0), hm.harmonic_index(l, 2 * l) + 1
                parts.append(torch.einsum("m,inm->in", self.clm[a:b], S[:, :, a:b] ** 2))  # Eq. 7
            if sz.l4:
                parts.append(four_body(S[:, :, 3:8]))
            if sz.l5:
                parts.append(five_body(S[:, :, 0:3]))
        return torch.cat(parts, -1)

    def atom_energies(self, p: dict, types, G: torch.Tensor) -> torch.Tensor:
        """E_i = sum_mu w1_mu tanh(sum_v W0_mu,v G_i,v + b0_mu) + b1 with the
        parameters of species type[i] (D1.1)."""
        ti = torch.as_tensor(types, dtype=torch.long)
        z = torch.einsum("nhd,nd->nh", p["W0"][ti], G) + p["b0"][ti]
        return (p["w1"][ti] * torch.tanh(z)).sum(-1) + p["b1"][ti]

    # -- one structure --------------------------------------------------------
    def neighbors(self, st):
        tilt = getattr(st, "tilt", None)
        return (neighbor_pairs(st.pos, st.box, self.sz.rc_rad, tilt32=tilt),
                neighbor_pairs(st.pos, st.box, self.sz.rc_ang, tilt32=tilt))

    def structure(self, theta: torch.Tensor, st, nbrs=None, create_graph=False, need_forces=True):
        """Per-atom energies, total energy, forces [n,3] and the 3x3 virial
        W = -dE/d(strain) of one structure."""
        pr, pa = nbrs if nbrs is not None else self.neighbors(st)
        p = unpack(self.sz, theta)
        n = st.n
        x = torch.tensor(np.asarray(st.pos, np.float32).astype(np.float64), dtype=DT, requires_grad=need_forces)
        strain = torch.zeros(3, 3, dtype=DT, requires_grad=need_forces)
        HS = torch.tensor(shift_vectors(st.box, getattr(st, "tilt", None)), dtype=DT)   # [27, 3]

        def vec(pairs):
            i, j, c = (torch.as_tensor(pairs[:, k]) for k in range(3))
            d = (x[j] - x[i]) + HS[c]
            # homogeneous deformation r -> (1 + strain) r of positions and box
            return d + d @ strain.T

        G = self.descriptors(p, st.types, n, pr, vec(pr), pa, vec(pa))
        Ei = self.atom_energies(p, st.types, G)
        E = Ei.sum()
        if not need_forces:
            return dict(Ei=Ei, E=E, G=G)
        gx, gs = torch.autograd.grad(E, (x, strain), create_graph=create_graph)
        return dict(Ei=Ei, E=E, G=G, F=-gx, W=-gs)

    # -- batch ----------------------------------------------------------------
    def predict(self, theta_np, structures, nbr_cache=None):
        """E(n), F (per structure [n,3]), W(n) in (xx,yy,zz,xy,yz,zx), per-atom
        energies and descriptors, all float64 numpy."""
        theta = torch.tensor(np.asarray(theta_np).astype(np.float64), dtype=DT)
        out = dict(E=[], F=[], W=[], Ei=[], G=[])
        for k, st in enumerate(structures):
            nb = nbr_cache[k] if nbr_cache is not None else None
            r = self.structure(theta, st, nb)
            out["E"].append(float(r["E"].detach()))
            out["F"].append(r["F"].detach().numpy())
            out["W"].append(voigt(r["W"].detach()).numpy())
            out["Ei"].append(r["Ei"].detach().numpy())
            out["G"].append(r["G"].detach().numpy())
        out["E"] = np.array(out["E"])
        out["W"] = np.array(out["W"]).reshape(-1, 6)
        return out

    def loss_and_grad(self, theta_np, structures, labels: dict, lam=(1.0, 1.0, 0.1),
                      need_grad=True, nbr_cache=None):
        """L = le*Le + lf*Lf + lv*Lv (Eq. 9) with
            Le = 1/N_str sum_n ((E(n) - E_tar(n)) / N_n)^2           (Eq. 10)
            Lf = 1/(3N) sum_{i,a} (F_ia - F_tar_ia)^2                (Eq. 11)
            Lv = 1/(6 N_str) sum_n sum_c ((W_c(n) - W_tar_c(n)) / N_n)^2 (Eq. 12)
        and its exact gradient.  labels: 'energy' [S] totals, 'force' list of
        [n,3] (or [N,3]), 'virial' [S,6] totals."""
        theta = torch.tensor(np.asarray(theta_np).astype(np.float64), dtype=DT,
                             requires_grad=need_grad)
        S = len(structures)
        N = sum(st.n for st in structures)
        le, lf, lv = lam
        Et = np.asarray(labels["energy"], np.float64)
        Wt = np.asarray(labels["virial"], np.float64).reshape(S, 6)
        Ft = labels["force"]
        if not isinstance(Ft, (list, tuple)):
            Ft = np.asarray(Ft, np.float64).reshape(-1, 3)
            offs = np.cumsum([0] + [st.n for st in structures])
            Ft = [Ft[offs[k]:offs[k + 1]] for k in range(S)]
        grad = torch.zeros(self.sz.n_params, dtype=DT)
        acc = np.zeros(3)
        for k, st in enumerate(structures):
            nb = nbr_cache[k] if nbr_cache is not None else None
            r = self.structure(theta, st, nb, create_graph=need_grad)
            nn = st.n
            e = (r["E"] - Et[k]) / nn
            Le = e * e / S
            Lf = ((r["F"] - torch.tensor(np.asarray(Ft[k], np.float64), dtype=DT)) ** 2).sum() / (3 * N)
            w = (voigt(r["W"]) - torch.tensor(Wt[k], dtype=DT)) / nn
            Lv = (w * w).sum() / (6 * S)
            Lk = le * Le + lf * Lf + lv * Lv
            acc += [float(Le.detach()), float(Lf.detach()), float(Lv.detach())]
            if need_grad:
                (g,) = torch.autograd.grad(Lk, theta)
                grad += g
        L = le * acc[0] + lf * acc[1] + lv * acc[2]
        return np.array([L, acc[0], acc[1], acc[2]]), grad.numpy()


    def cotangent_grad(self, theta_np, structures, e_bar, f_bar, v_bar, nbr_cache=None):
        """Gradient of sum_n e_bar[n] E(n) + sum_i f_bar_i . F_i + sum_n v_bar[n] . W(n)
        with respect to the parameters (a vector-Jacobian product written as the
        derivative of that contraction).  f_bar: list of [n,3] or [N,3]."""
        theta = torch.tensor(np.asarray(theta_np).astype(np.float64), dtype=DT, requires_grad=True)
        S = len(structures)
        e_bar = np.asarray(e_bar, np.float64)
        v_bar = np.asarray(v_bar, np.float64).reshape(S, 6)
        if not isinstance(f_bar, (list, tuple)):
            fb = np.asarray(f_bar, np.float64).reshape(-1, 3)
            offs = np.cumsum([0] + [st.n for st in structures])
            f_bar = [fb[offs[k]:offs[k + 1]] for k in range(S)]
        grad = torch.zeros(self.sz.n_params, dtype=DT)
        for k, st in enumerate(structures):
            nb = nbr_cache[k] if nbr_cache is not None else None
            r = self.structure(theta, st, nb, create_graph=True)
            c = (e_bar[k] * r["E"] + (torch.tensor(np.asarray(f_bar[k], np.float64), dtype=DT) * r["F"]).sum()
                 + (torch.tensor(v_bar[k], dtype=DT) * voigt(r["W"])).sum())
            (g,) = torch.autograd.grad(c, theta)
            grad += g
        return grad.numpy()


def four_body(S2: torch.Tensor) -> torch.Tensor:
    """q4_n = tr(M_n^3) with M_n the traceless symmetric matrix that the l = 2
    sums S_n2m represent: M_zz = S_20/3, M_xz = S_21, M_yz = S_22,
    M_xx - M_yy = S_23, M_xy = S_24/2 (the l = 2 harmonics of Appendix B are
    the components of u u^T - I/3).  The paper names the 4-body term without
    defining it; a cubic rotation invariant of the l = 2 sums is unique up to
    scale, and this is the unit-scale one."""
    s0, s1, s2, s3, s4 = (S2[..., m] for m in range(5))
    mzz = s0 / 3
    mxx = -s0 / 6 + s3 / 2
    myy = -s0 / 6 - s3 / 2
    mxy = s4 / 2
    M = torch.stack([torch.stack([mxx, mxy, s1], -1),
                     torch.stack([mxy, myy, s2], -1),
                     torch.stack([s1, s2, mzz], -1)], -2)
    return torch.einsum("...ab,...bc,...ca->...", M, M, M)


def five_body(S1: torch.Tensor) -> torch.Tensor:
    """q5_n = (sum_m S_n1m^2)^2, the quartic rotation invariant of the l = 1
    sums (unique up to scale; the paper names the 5-body term only)."""
    return (S1 ** 2).sum(-1) ** 2


def voigt(W: torch.Tensor) -> torch.Tensor:
    """(xx, yy, zz, xy, yz, zx) components of a 3x3 virial."""
    return torch.stack([W[0, 0], W[1, 1], W[2, 2], W[0, 1], W[1, 2], W[2, 0]])


# ----------------------------------------------------------------------------
# optimizer and schedule
# ----------------------------------------------------------------------------
def adam_step(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Bias-corrected Adam (the optimizer the paper adopts, Sec. I), float64.
    `step` is 1-based.  Returns new (theta, m, v)."""
    theta, m, v, g = (np.asarray(a, np.float64) for a in (theta, m, v, g))
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def lr_schedule(s: int, lr_start: float, lr_stop: float, n_warmup: int, n_total: int) -> float:
    """Eq. 17: linear warmup from lr_stop to lr_start over n_warmup steps,
    then cosine decay back to lr_stop at n_total."""
    if s < n_warmup:
        return lr_stop + s / n_warmup * (lr_start - lr_stop)
    frac = (s - n_warmup) / max(n_total - n_warmup, 1)
    frac = min(frac, 1.0)
    return lr_stop + (lr_start - lr_stop) * 0.5 * (1 + math.cos(math.pi * frac))
