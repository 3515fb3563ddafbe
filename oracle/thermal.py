"""Steady-state heat equation and the self-consistent field <-> temperature loop,
in FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Model (Sec. 2.2):
  k lap T + q = 0,   q = sum_j alpha_j I_j + beta_j I_j^2,   I_j = eps0 c n_j |A_j|^2 / 2
with a constant conductivity k.  Faces touching the oven are held at T_oven
(Dirichlet); faces in air lose heat by convection, -k dT/dn = h (T - T_inf),
with n the outward normal; an insulated face is a convective face with h = 0.

Discretisation (Sec. 3.2, the second-order finite-difference equation of the
heat equation):
  * the nodes are those of the SSFM grid: transverse nodes are the field
    samples x_m = (m - nx/2) dx, m = 0..nx-1 (likewise y), so the x faces of the
    crystal sit at the first and last sample; z nodes are z_l = l dz, l = 0..nz,
    with faces at z = 0 and z = L;
  * every node that is not on an oven face obeys the 7-point equation
    sum_d (T_{+d} - 2 T + T_{-d}) / h_d^2 = -q / k;
    on a convective face the missing outside neighbour is eliminated through
    the central difference of the boundary condition,
    T_outside = T_inside_neighbour - 2 h_d (h / k) (T - T_inf);
    nodes on an oven face (edges and corners included) are T_oven.

Coupling to the march (Sec. 2.2 and the flowchart of Sec. 4):
  * the heat source at node l uses the fields at the step boundary z_l;
  * the march takes T at each step's mid-plane, T_mid[s] = (T[s] + T[s+1]) / 2;
  * loop: q = 0 -> T -> march with T -> q -> T -> ... until the largest change
    of T between two iterations is at most tol.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .ssfm import EPS0, C_LIGHT, coefficients, propagate

FACES = ("x-", "x+", "y-", "y+", "z-", "z+")


@dataclass
class ThermalParams:
    k_th: float                     # thermal conductivity [W/(m K)]
    h_conv: float                   # convection coefficient [W/(m^2 K)]
    t_inf: float                    # air temperature [K]
    t_oven: float                   # oven temperature [K]
    faces: Dict[str, str] = field(default_factory=dict)   # face -> "oven" | "air" | "insulated"

    def face(self, name: str) -> str:
        return self.faces.get(name, "air")


def bottom_oven(k_th, h_conv, t_inf, t_oven) -> ThermalParams:
    """Crystal resting on an oven along its bottom face y-; the rest in air."""
    return ThermalParams(k_th, h_conv, t_inf, t_oven, {"y-": "oven"})


def surrounding_oven(k_th, h_conv, t_inf, t_oven) -> ThermalParams:
    """Oven around the four long faces; the two end faces in air."""
    return ThermalParams(k_th, h_conv, t_inf, t_oven,
                         {"x-": "oven", "x+": "oven", "y-": "oven", "y+": "oven"})


def grid_shape(p: dict):
    """(nz + 1, ny, nx) nodes."""
    return p["nz"] + 1, p["ny"], p["nx"]


def steps(p: dict):
    """Node spacings (dx, dy, dz)."""
    return p["lx"] / p["nx"], p["ly"] / p["ny"], p["lcr"] / p["nz"]


def oven_mask(p: dict, tp: ThermalParams) -> np.ndarray:
    """True at nodes held at T_oven."""
    nzn, ny, nx = grid_shape(p)
    m = np.zeros((nzn, ny, nx), dtype=bool)
    if tp.face("x-") == "oven":
        m[:, :, 0] = True
    if tp.face("x+") == "oven":
        m[:, :, -1] = True
    if tp.face("y-") == "oven":
        m[:, 0, :] = True
    if tp.face("y+") == "oven":
        m[:, -1, :] = True
    if tp.face("z-") == "oven":
        m[0, :, :] = True
    if tp.face("z+") == "oven":
        m[-1, :, :] = True
    return m


def system(p: dict, tp: ThermalParams, q: np.ndarray):
    """Sparse matrix and right-hand side of the node equations of the free
    (non-oven) nodes, with the oven temperatures moved to the right-hand side.
    q: [nz+1, ny, nx] heat source [W/m^3].  Returns (A, rhs, free_mask)."""
    nzn, ny, nx = grid_shape(p)
    hs = steps(p)
    dims = (nx, ny, nzn)                      # sizes along x, y, z
    strides = (1, nx, nx * ny)
    names = (("x-", "x+"), ("y-", "y+"), ("z-", "z+"))
    n = nx * ny * nzn
    oven = oven_mask(p, tp).ravel()
    beta = tp.h_conv / tp.k_th
    rows, cols, vals = [], [], []
    rhs = -np.asarray(q, dtype=np.float64).ravel() / tp.k_th
    idx = np.arange(n)
    coord = (idx % nx, (idx // nx) % ny, idx // (nx * ny))
    for d in range(3):
        h = hs[d]
        i = coord[d]
        st = strides[d]
        lo, hi = i == 0, i == dims[d] - 1
        mid = ~lo & ~hi
        # interior direction: (T+ - 2T + T-) / h^2
        r = idx[mid]
        for o in (st, -st):
            rows.append(r)
            cols.append(r + o)
            vals.append(np.full(r.size, 1.0 / h ** 2))
        rows.append(r)
        cols.append(r)
        vals.append(np.full(r.size, -2.0 / h ** 2))
        # boundary nodes: outside neighbour eliminated through the face condition
        for sel, inward, face in ((lo, st, names[d][0]), (hi, -st, names[d][1])):
            r = idx[sel]
            b = 0.0 if tp.face(face) == "insulated" else beta
            rows.append(r)
            cols.append(r + inward)
            vals.append(np.full(r.size, 2.0 / h ** 2))
            rows.append(r)
            cols.append(r)
            vals.append(np.full(r.size, -2.0 / h ** 2 - 2.0 * b / h))
            rhs[r] -= 2.0 * b / h * tp.t_inf
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    full = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    free = ~oven
    a = full[free][:, free]
    rhs_free = rhs[free] - full[free][:, oven] @ np.full(int(oven.sum()), tp.t_oven)
    return a, rhs_free, free


def solve(p: dict, tp: ThermalParams, q: np.ndarray) -> np.ndarray:
    """Node temperatures [nz+1, ny, nx] by a sparse direct solve."""
    a, rhs, free = system(p, tp, q)
    t = np.full(free.size, tp.t_oven)
    t[free] = spla.spsolve(a.tocsc(), rhs)
    return t.reshape(grid_shape(p))


def heat_source(p: dict, a_f: np.ndarray, a_sh: np.ndarray) -> np.ndarray:
    """q = sum_j alpha_j I_j + beta_j I_j^2 on one plane of nodes (Sec. 2.2)."""
    i_f = EPS0 * C_LIGHT * p["n_f"] / 2.0 * np.abs(a_f) ** 2
    i_sh = EPS0 * C_LIGHT * p["n_sh"] / 2.0 * np.abs(a_sh) ** 2
    return (p["alpha_f"] * i_f + p["beta_f"] * i_f ** 2
            + p["alpha_sh"] * i_sh + p["beta_sh"] * i_sh ** 2)


def march_heat(p: dict, a_f0, a_sh0, dk_z=None, temp=None):
    """Forward march that also returns the heat source at every z node."""
    out = propagate(p, a_f0, a_sh0, dk_z=dk_z, temp=temp, return_states=True)
    planes = [heat_source(p, a, b) for a, b in out["states"]]
    planes.append(heat_source(p, out["a_f"], out["a_sh"]))
    out["q"] = np.stack(planes)
    return out


def midplanes(t_nodes: np.ndarray) -> np.ndarray:
    """T at the step mid-planes, [nz, ny, nx]."""
    return 0.5 * (t_nodes[1:] + t_nodes[:-1])


def self_consistent(p: dict, tp: ThermalParams, a_f0, a_sh0, dk_z=None, tol: float = 1e-6,
                    max_iter: int = 30):
    """The fixed-point loop of the flowchart.  Returns the final node
    temperatures, the last march, and the history of max |T_new - T_old|."""
    shape = grid_shape(p)
    t = solve(p, tp, np.zeros(shape))
    hist = []
    march = None
    for _ in range(max_iter):
        march = march_heat(p, a_f0, a_sh0, dk_z=dk_z, temp=midplanes(t))
        t_new = solve(p, tp, march["q"])
        hist.append(float(np.max(np.abs(t_new - t))))
        t = t_new
        if hist[-1] <= tol:
            break
    return t, march, hist


def energy_balance(p: dict, tp: ThermalParams, t: np.ndarray, q: np.ndarray):
    """Discrete energy balance of a solution t for source q.

    Each free node owns a control volume dx dy dz, halved once for every face it
    lies on.  Summing k (node equation) x volume over the free nodes, the
    exchange terms between free neighbours cancel in pairs, leaving
      source = sum_free q V
      loss   = sum over air faces of h (T - T_inf) dA
             + sum over free-oven neighbour pairs of k (T_free - T_oven) / h_d^2 V_free
    which must be equal.  Returns (source, loss) in W."""
    nzn, ny, nx = grid_shape(p)
    dx, dy, dz = steps(p)
    hs = {2: dx, 1: dy, 0: dz}
    names = {2: ("x-", "x+"), 1: ("y-", "y+"), 0: ("z-", "z+")}
    w = np.ones(t.shape)
    for ax in (0, 1, 2):
        for end in (0, t.shape[ax] - 1):
            sl = [slice(None)] * 3
            sl[ax] = end
            w[tuple(sl)] *= 0.5
    vol = w * dx * dy * dz
    oven = oven_mask(p, tp)
    free = ~oven
    source = float(np.sum((q * vol)[free]))
    loss = 0.0
    for ax in (0, 1, 2):
        h = hs[ax]
        for end, name, inward in ((0, names[ax][0], 1), (t.shape[ax] - 1, names[ax][1], -1)):
            sl = [slice(None)] * 3
            sl[ax] = end
            sl = tuple(sl)
            if tp.face(name) == "air":
                # dA = 2 V / h for a node on this face
                loss += float(np.sum((tp.h_conv * (t[sl] - tp.t_inf) * 2.0 * vol[sl] / h)[free[sl]]))
            elif tp.face(name) == "oven":
                # free nodes next to this oven face
                nb = [slice(None)] * 3
                nb[ax] = end + inward
                nb = tuple(nb)
                pair = free[nb]
                loss += float(np.sum((tp.k_th * (t[nb] - t[sl]) / h ** 2 * vol[nb])[pair]))
    return source, loss
