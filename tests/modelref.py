"""Independent numpy statements of model quantities used to pin the oracle.

These are written directly from the free-energy functional and the
concentration definition (Sec. 2 of the paper), not from the oracle's
flux-and-update code, so that a dropped term, a wrong sign or a wrong index in
the oracle's time step shows up as a disagreement.
"""
from __future__ import annotations

import math

import numpy as np

LIQ = 3


def T_of(p, nz, t, dx=1.0):
    k = np.arange(nz, dtype=np.float64)
    return p["T0"] + p["G"] * (k * dx + p["zoff"] - p["v"] * t)


def conc_total_field(p, phi, mu, t, dx=1.0):
    """c_i(x) = sum_a h_a(phi) (chi_ai(T) mu_i + cbar_ai(T)), h = phi^2/sum phi^2."""
    nz = phi.shape[1]
    T = T_of(p, nz, t, dx)[:, None, None]
    S = (phi ** 2).sum(axis=0)
    out = []
    for i in range(2):
        c = np.zeros_like(S)
        for a in range(4):
            chi = p["chi0"][a][i] + p["chi1"][a][i] * (T - p["TE"])
            cb = p["c0"][a][i] + p["c1"][a][i] * (T - p["TE"])
            c = c + (phi[a] ** 2 / S) * (chi * mu[i] + cb)
        out.append(c)
    return np.stack(out)


def energy_terms(p, phi, mu, T, dx=1.0):
    """All additive terms of the isotropic discrete energy with uniform T:

    E_h = dx^3 [ sum_faces eps T sum_{a<b} gamma_ab (q_ab . e_d)^2
               + sum_cells ( (T/eps) omega(phi) + sum_b h_b psi_b(mu, T) ) ]

    with face quantities q_ab.e_d = pbar_a d_d phi_b - pbar_b d_d phi_a
    (pbar = face average, d_d = normal difference), periodic faces in x and y,
    and no faces across the z boundaries.  Returned as a flat array so the
    caller can sum it exactly (math.fsum)."""
    eps = p["eps"]
    g = np.array(p["gamma"])
    terms = []
    for d in range(3):
        axis = 3 - d  # array axes: (a, z, y, x)
        if d == 2:
            L = phi[:, :-1]
            U = phi[:, 1:]
        else:
            L = phi
            U = np.roll(phi, -1, axis=axis)
        pb = 0.5 * (L + U)
        dd = (U - L) / dx
        face = np.zeros(L.shape[1:])
        for a in range(4):
            for b in range(a + 1, 4):
                q = pb[a] * dd[b] - pb[b] * dd[a]
                face = face + g[a][b] * q * q
        terms.append((dx ** 3) * eps * T * face.ravel())
    k16 = 16.0 / math.pi ** 2
    om = np.zeros(phi.shape[1:])
    for a in range(4):
        for b in range(a + 1, 4):
            om = om + k16 * g[a][b] * phi[a] * phi[b]
            for c in range(b + 1, 4):
                om = om + p["gamma3"] * phi[a] * phi[b] * phi[c]
    S = (phi ** 2).sum(axis=0)
    psi_mix = np.zeros_like(S)
    for a in range(4):
        chi = [p["chi0"][a][i] + p["chi1"][a][i] * (T - p["TE"]) for i in range(2)]
        cb = [p["c0"][a][i] + p["c1"][a][i] * (T - p["TE"]) for i in range(2)]
        wb = p["w0"][a] + p["w1"][a] * (T - p["TE"])
        psi_a = (-0.5 * (chi[0] * mu[0] ** 2 + chi[1] * mu[1] ** 2)
                 - (cb[0] * mu[0] + cb[1] * mu[1]) + wb)
        psi_mix = psi_mix + (phi[a] ** 2 / S) * psi_a
    terms.append((dx ** 3) * ((T / eps) * om + psi_mix).ravel())
    return np.concatenate(terms)


def energy(p, phi, mu, T, dx=1.0):
    return math.fsum(energy_terms(p, phi, mu, T, dx))


def _val(f, k, j, i):
    nz, ny, nx = f.shape
    k = min(max(k, 0), nz - 1)  # zero-gradient mirror in z
    return f[k, j % ny, i % nx]


def face_gradient_vec(f, i, j, k, d, dx=1.0):
    """Normal difference and 4-point tangential averages at face (i,j,k)+e_d/2."""
    e = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    iu, ju, ku = i + e[d][0], j + e[d][1], k + e[d][2]
    g = np.zeros(3)
    g[d] = (_val(f, ku, ju, iu) - _val(f, k, j, i)) / dx
    for t in range(3):
        if t == d:
            continue
        s = e[t]
        plus = _val(f, k + s[2], j + s[1], i + s[0]) + _val(f, ku + s[2], ju + s[1], iu + s[0])
        minus = _val(f, k - s[2], j - s[1], i - s[0]) + _val(f, ku - s[2], ju - s[1], iu - s[0])
        g[t] = (plus - minus) / (4.0 * dx)
    return g


def antitrap_matrix_literal(p, phi0, phi1, mu, i, j, k, d, Tf, dx=1.0):
    """Eq. (4) evaluated literally on one face with an explicit dyadic
    product: J = (pi eps/4) sum_{a != l} g_a h_l / sqrt(phi_a phi_l) dphi_a/dt
    (n_a . n_l) (c^l - c^a) (x) n_a, with g_a = phi_a, h_l = phi_l^2/sum phi^2,
    phi taken as the face average and dphi/dt as the face-averaged difference
    quotient.  Needs phi strictly inside the simplex.  Returns the 2x3 matrix."""
    e = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    iu, ju, ku = i + e[d][0], j + e[d][1], k + e[d][2]
    pb = np.array([0.5 * (_val(phi0[a], k, j, i) + _val(phi0[a], ku, ju, iu)) for a in range(4)])
    rate = np.array([0.5 * ((_val(phi1[a], k, j, i) - _val(phi0[a], k, j, i))
                            + (_val(phi1[a], ku, ju, iu) - _val(phi0[a], ku, ju, iu))) / p["dt"]
                     for a in range(4)])
    mb = np.array([0.5 * (_val(mu[q], k, j, i) + _val(mu[q], ku, ju, iu)) for q in range(2)])
    grads = [face_gradient_vec(phi0[a], i, j, k, d, dx) for a in range(4)]
    n = [g / np.linalg.norm(g) for g in grads]

    def conc(a):
        return np.array([(p["chi0"][a][q] + p["chi1"][a][q] * (Tf - p["TE"])) * mb[q]
                         + p["c0"][a][q] + p["c1"][a][q] * (Tf - p["TE"]) for q in range(2)])

    hl = pb[LIQ] ** 2 / np.sum(pb ** 2)
    J = np.zeros((2, 3))
    for a in range(3):
        weight = pb[a] * hl / math.sqrt(pb[a] * pb[LIQ])
        J += weight * rate[a] * float(np.dot(n[a], n[LIQ])) * np.outer(conc(LIQ) - conc(a), n[a])
    return (math.pi * p["eps"] / 4.0) * J
