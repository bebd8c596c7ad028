"""A second, deliberately naive implementation of one time step, used to pin the oracle.

Where the oracle collides in moment space with the closed forms of Eqs. 21-23
and 36-37, this version works in population space: it builds f^eq from Eq. 11,
R_i from Eq. 15, F_i from Eq. 14, g^eq from Eqs. 25-26, T_i from Eq. 29 and G_i
from Eq. 27, and applies the dense matrices M^-1 S M and M^-1 (I - S/2) M of
Eqs. 10, 14, 24 and 27 with a numerically inverted M read from the printed
matrix (tests/golden/d2q9_matrix_M.txt).  The lattice comes from the cos/sin
formula of Eq. 12.  Propagation is written as a push (each post-collision
population moves to x + c_i and is reflected where it would leave the grid),
the mirror of the oracle's pull.  Velocity comes from solving Eq. 31 together
with Eq. 30 as a 2x2 linear system.  Only for grids of a few dozen nodes.

collision = "nmrt" (the non-orthogonal extension named in Sec. 4) replaces M
by the raw-moment basis built from the lattice monomials, each raw row taking
the rate of the orthogonal moment it stands for, and uses the pressure
coefficient that the Chapman-Enskog step of Appendix C gives for that basis.
"""
from __future__ import annotations

import math
import os

import numpy as np

_GOLD = os.path.join(os.path.dirname(__file__), "golden")


def printed_M() -> np.ndarray:
    rows = [l.split() for l in open(os.path.join(_GOLD, "d2q9_matrix_M.txt"))
            if l.strip() and not l.startswith("#")]
    return np.array(rows, dtype=np.float64)


def lattice_eq12():
    """c_i from the cos/sin formula of Eq. 12 (x -> z, y -> r); weights of Sec. 2.2."""
    c = [(0.0, 0.0)]
    for i in range(1, 5):
        a = (i - 1) * math.pi / 2
        c.append((math.cos(a), math.sin(a)))
    for i in range(5, 9):
        a = (i - 5) * math.pi / 2 + math.pi / 4
        c.append((math.sqrt(2) * math.cos(a), math.sqrt(2) * math.sin(a)))
    c = np.rint(np.array(c)).astype(int)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    return c[:, 0], c[:, 1], w


CZ, CR, WT = lattice_eq12()
CS2 = 1.0 / 3.0
MM = printed_M()
MINV = np.linalg.inv(MM)

# non-orthogonal (raw-moment) basis of the extension named in Sec. 4: rows
# 1, c_z, c_r, c_z^2 + c_r^2, c_z^2 - c_r^2, c_z c_r, c_z^2 c_r, c_z c_r^2, c_z^2 c_r^2
RAW = np.array([np.ones(9), CZ, CR, CZ**2 + CR**2, CZ**2 - CR**2, CZ * CR, CZ**2 * CR, CZ * CR**2,
                CZ**2 * CR**2], dtype=np.float64)
RAWINV = np.linalg.inv(RAW)
# the orthogonal moment (row of M) whose rate each raw row takes:
# 1 <- rho, c_z <- j_z, c_r <- j_r, c^2 <- e, c_z^2 - c_r^2 <- p_zz, c_z c_r <- p_zr,
# c_z^2 c_r <- q_r, c_z c_r^2 <- q_z, c_z^2 c_r^2 <- eps
RAW_RATE = [0, 3, 5, 1, 7, 8, 6, 4, 2]


def _ghost_index(nr, nz, zper, k, j):
    if j < 0:
        j = -1 - j
    if j >= nr:
        j = 2 * nr - 1 - j
    if zper:
        k = k % nz
    else:
        if k < 0:
            k = -1 - k
        if k >= nz:
            k = 2 * nz - 1 - k
    return k, j


def grad_lap(chi, zper):
    """Eqs. 39-40 with the ghost rules, node by node."""
    nr, nz = chi.shape
    gz = np.zeros_like(chi)
    gr = np.zeros_like(chi)
    lap = np.zeros_like(chi)
    for j in range(nr):
        for k in range(nz):
            for i in range(1, 9):
                k1, j1 = _ghost_index(nr, nz, zper, k + CZ[i], j + CR[i])
                k2, j2 = _ghost_index(nr, nz, zper, k + 2 * CZ[i], j + 2 * CR[i])
                t = 8 * chi[j1, k1] - chi[j2, k2]
                gz[j, k] += WT[i] * CZ[i] * t / (6 * CS2)
                gr[j, k] += WT[i] * CR[i] * t / (6 * CS2)
                lap[j, k] += WT[i] * (16 * chi[j1, k1] - chi[j2, k2] - 15 * chi[j, k]) / (6 * CS2)
    return gz, gr, lap


def push_stream(post, zper):
    """Propagation (Eq. 20) as a push, reflecting at the axis and bouncing back at walls."""
    _, nr, nz = post.shape
    out = np.full_like(post, np.nan)
    opp = [int(np.where((CZ == -CZ[i]) & (CR == -CR[i]))[0][0]) for i in range(9)]
    mir = [int(np.where((CZ == CZ[i]) & (CR == -CR[i]))[0][0]) for i in range(9)]
    for i in range(9):
        for j in range(nr):
            for k in range(nz):
                tk, tj = k + CZ[i], j + CR[i]
                hits_wall = tj >= nr
                if zper:
                    tk %= nz
                elif tk < 0 or tk >= nz:
                    hits_wall = True
                if hits_wall:
                    out[opp[i], j, k] = post[i, j, k]
                elif tj < 0:
                    out[mir[i], 0, tk] = post[i, j, k]
                else:
                    out[i, tj, tk] = post[i, j, k]
    assert np.isfinite(out).all()
    return out


def naive_step(spec, f, g, aux, t=0):
    """One step from post-propagation (f, g) and previous (phi, u_z, u_r) at time t.

    Returns (f_new, g_new, aux_new, fields) with fields holding phi, rho, p, u_z, u_r.
    spec.g_ramp > 0: the acceleration is g_z (t + 1) / g_ramp while t + 1 < g_ramp.
    spec.free_s1: the energy moment relaxes at spec.s_g[1] instead of 1/tau_g.
    """
    nr, nz = f.shape[1:]
    zper = bool(spec.z_periodic)
    r = (np.arange(nr) + 0.5)[:, None] * np.ones((1, nz))
    phi = f.sum(0) / r                                                     # Eq. 16
    rho = phi * spec.rho_l + (1 - phi) * spec.rho_g                        # Eq. 17
    nu = phi * spec.nu_l + (1 - phi) * spec.nu_g                           # Eq. 35
    gz, gr, lap = grad_lap(phi, zper)
    rgz, rgr, _ = grad_lap(rho, zper)
    kap, beta = 1.5 * spec.sigma * spec.W, 12 * spec.sigma / spec.W
    tau_f = spec.mobility / CS2 + 0.5                                      # Eq. 18
    ramp = float(getattr(spec, "g_ramp", 0.0))
    g_acc = spec.g_z * ((t + 1) / ramp) if ramp > 0 and t + 1 < ramp else spec.g_z
    free_s1 = bool(getattr(spec, "free_s1", False))
    form = getattr(spec, "collision", "mrt")
    srt = form == "srt"                                   # every rate 1/tau (end of Sec. 2.2)
    # basis of the collision: the printed M, or the raw moments (Sec. 4)
    B, BINV = (RAW, RAWINV) if form == "nmrt" else (MM, MINV)

    def in_basis(rates):
        return np.diag([rates[a] for a in RAW_RATE]) if form == "nmrt" else np.diag(rates)

    Sf = in_basis([spec.s_f[0], spec.s_f[1], spec.s_f[2], 1 / tau_f, 1 / tau_f, 1 / tau_f,
                   1 / tau_f, spec.s_f[7], spec.s_f[8]])
    if srt:
        Sf = np.eye(9) / tau_f
    fpost = np.empty_like(f)
    gpost = np.empty_like(g)
    aux_new = np.empty_like(aux)
    fields = {k: np.empty((nr, nz)) for k in ("phi", "rho", "p", "uz", "ur")}
    for j in range(nr):
        for k in range(nz):
            rr = r[j, k]
            ph, rh, nv = phi[j, k], rho[j, k], nu[j, k]
            mu = 4 * beta * ph * (ph - 1) * (ph - 0.5) - kap * lap[j, k]       # Eq. 4
            mut = mu - kap * gr[j, k] / rr
            Fs = np.array([mut * gz[j, k], mut * gr[j, k]])
            G = np.array([(rh - spec.rho_l) * g_acc, 0.0])
            tau_g = nv / CS2 + 0.5                                            # Eq. 34
            s_nu = 1 / tau_g
            s1 = spec.s_g[1] if free_s1 else s_nu
            Sg = in_basis([spec.s_g[0], s1, spec.s_g[2], spec.s_g[3], spec.s_g[4], spec.s_g[5],
                           spec.s_g[6], s_nu, s_nu])
            s2 = spec.s_g[2]
            if srt:
                Sg = np.eye(9) * s_nu
                s1 = s2 = s_nu
            sp = (s1 + s2 - s1 * s2) / (2 * s1 * s2)
            if form == "nmrt":
                # the rho u_r coefficient of g_0 - g_0^eq for the raw basis
                # (tests/test_oracle_pins.py derives both forms)
                sp = 0.5 * (3 / s1 - 1 / s2 - 1)
            up = aux[1:, j, k]
            gv = g[:, j, k]
            s0 = WT[0] * (-(up @ up) / (2 * CS2))
            p = CS2 / (1 - WT[0]) * (gv[1:].sum() / rr + 0.5 * (up[0] * rgz[j, k] + up[1] * rgr[j, k])
                                     + rh * s0 - sp * WT[0] * rh * up[1] / rr)      # Eq. 33
            # Eq. 31 with F of Eq. 30: r rho u = sum c g + F/2, F_r containing -2 rho nu u_r / r
            A = np.array([[rr * rh, 0.0], [0.0, rr * rh + 0.5 * 2 * rh * nv / rr]])
            b = np.array([CZ @ gv, CR @ gv]) + 0.5 * (rr * (Fs + G) + np.array([0.0, p]))
            u = np.linalg.solve(A, b)
            F = rr * (Fs + G) + np.array([0.0, p - 2 * rh * nv * u[1] / rr])

            # ---- f: Eqs. 11, 14, 15, 19 in population space
            J = np.array([rr * ph * u[0], rr * ph * u[1] + spec.mobility * ph])
            php = aux[0, j, k]
            Jp = np.array([rr * php * aux[1, j, k], rr * php * aux[2, j, k] + spec.mobility * php])
            lam = -4 * (ph - 1) * ph / spec.W
            gm = math.hypot(gz[j, k], gr[j, k])
            n = np.array([gz[j, k], gr[j, k]]) / gm if gm > 1e-12 else np.zeros(2)
            feq = np.array([WT[i] * (rr * ph + (CZ[i] * J[0] + CR[i] * J[1]) / CS2) for i in range(9)])
            vec = (J - Jp) + CS2 * rr * n * lam
            R = np.array([WT[i] * (CZ[i] * vec[0] + CR[i] * vec[1]) / CS2 for i in range(9)])
            Fi = BINV @ (np.eye(9) - Sf / 2) @ B @ R
            fpost[:, j, k] = f[:, j, k] - BINV @ Sf @ B @ (f[:, j, k] - feq) + Fi

            # ---- g: Eqs. 24-29 in population space
            def s_i(i):
                cu = CZ[i] * u[0] + CR[i] * u[1]
                return WT[i] * (cu / CS2 + cu * cu / (2 * CS2 * CS2) - (u @ u) / (2 * CS2))
            geq = np.array([rr * p / CS2 * (WT[i] - (1 if i == 0 else 0)) + rr * rh * s_i(i)
                            for i in range(9)])
            drr = np.array([rr * rgz[j, k], rr * rgr[j, k] + rh])   # d_beta (r rho)
            T = np.empty(9)
            for i in range(9):
                c = np.array([CZ[i], CR[i]])
                T[i] = WT[i] * ((c @ F) / CS2 + (u @ c) * (c @ drr) / CS2 - rh * u[1])
            Gi = BINV @ (np.eye(9) - Sg / 2) @ B @ T
            gpost[:, j, k] = gv - BINV @ Sg @ B @ (gv - geq) + Gi
            aux_new[:, j, k] = (ph, u[0], u[1])
            fields["phi"][j, k], fields["rho"][j, k], fields["p"][j, k] = ph, rh, p
            fields["uz"][j, k], fields["ur"][j, k] = u
    return push_stream(fpost, zper), push_stream(gpost, zper), aux_new, fields
