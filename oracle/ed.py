"""Exact diagonalisation of H_eta for the hard-core Bose-Hubbard model.

TEST INFRASTRUCTURE ONLY: thermal expectation values that pin the oracle.

    H     = sum_<ij> [ -t (b_i^+ b_j + h.c.) + V n_i n_j ] - mu sum_i n_i
    H_eta = H - eta sum_i (b_i + b_i^+)

(model of Eq. (BH) with the per-bond reading of its garbled sums, and the
fictitious source term of the paper's introduction).  Hard-core bosons map
to spin 1/2: b_i + b_i^+ is sigma^x on site i.

Two solvers:
  * ``thermal_dense``   -- the full matrix, numpy ``eigh`` (N <= 12 sites);
  * ``thermal_sectors`` -- block diagonal in lattice momentum (the model is
    translation invariant; eta breaks particle number but not translations),
    used for the 4x4 lattice (2^16 states, 16 blocks).

Returned per-site observables: E = <H>/N, E_eta = <H_eta>/N, n = <n_i>,
Q = <sum_i (b_i + b_i^+)>/N, nn = <sum_<ij> n_i n_j>/N, K = <-t sum hop>/N.
"""
from __future__ import annotations

import numpy as np


def lattice_bonds(Lx: int, Ly: int):
    bonds = []
    for y in range(Ly):
        for x in range(Lx):
            s = y * Lx + x
            bonds.append((s, y * Lx + (x + 1) % Lx))
            bonds.append((s, ((y + 1) % Ly) * Lx + x))
    return bonds


def _diag_parts(Lx, Ly, states):
    N = Lx * Ly
    occ = ((states[:, None] >> np.arange(N)) & 1).astype(np.float64)
    nsum = occ.sum(axis=1)
    nn = np.zeros(len(states))
    for a, c in lattice_bonds(Lx, Ly):
        nn += occ[:, a] * occ[:, c]
    return nsum, nn


def hamiltonian_dense(Lx, Ly, t, V, mu, eta):
    """Return (H_eta, Q, diag_n, diag_nn, hop) as dense matrices / vectors."""
    N = Lx * Ly
    dim = 1 << N
    states = np.arange(dim, dtype=np.int64)
    nsum, nn = _diag_parts(Lx, Ly, states)
    hop = np.zeros((dim, dim))
    for a, c in lattice_bonds(Lx, Ly):
        na = (states >> a) & 1
        nc = (states >> c) & 1
        m = na != nc
        src = states[m]
        dst = src ^ ((1 << a) | (1 << c))
        hop[dst, src] += -t
    Q = np.zeros((dim, dim))
    for i in range(N):
        Q[states ^ (1 << i), states] += 1.0
    H = hop + np.diag(V * nn - mu * nsum)
    return H - eta * Q, Q, nsum, nn, hop


def _thermal(evals, evecs, beta, ops_diag, ops_full):
    w = np.exp(-beta * (evals - evals.min()))
    Z = w.sum()
    out = {}
    prob = np.abs(evecs) ** 2
    for name, d in ops_diag.items():
        out[name] = float((w * (d @ prob)).sum() / Z)
    for name, M in ops_full.items():
        dm = np.real(np.einsum("in,in->n", evecs.conj(), M @ evecs))
        out[name] = float((w * dm).sum() / Z)
    out["E_eta_total"] = float((w * evals).sum() / Z)
    return out


def thermal_dense(Lx, Ly, beta, t, V, mu, eta):
    N = Lx * Ly
    H, Q, nsum, nn, hop = hamiltonian_dense(Lx, Ly, t, V, mu, eta)
    evals, evecs = np.linalg.eigh(H)
    r = _thermal(evals, evecs, beta, {"n": nsum, "nn": nn}, {"Q": Q, "K": hop})
    return _finish(r, N, V, mu, eta)


def green_dense(Lx, Ly, beta, t, V, mu, eta, disps):
    """<T (b_j + b_j^+)(tau) (b_i + b_i^+)(0)> = Tr(e^{-(beta-tau) H} X_j
    e^{-tau H} X_i) / Z (X = sigma^x, H = H_eta), averaged over sites i with
    j = i + (rx, ry), for each displacement (rx, ry) or (rx, ry, tau)."""
    N = Lx * Ly
    H, _, _, _, _ = hamiltonian_dense(Lx, Ly, t, V, mu, eta)
    evals, evecs = np.linalg.eigh(H)
    e = evals - evals.min()
    Z = np.exp(-beta * e).sum()
    states = np.arange(1 << N, dtype=np.int64)
    # sigma^x_i in the eigenbasis
    X = []
    for i in range(N):
        X.append(evecs.T @ evecs[states ^ (1 << i), :])
    out = []
    for dd in disps:
        rx, ry = dd[0], dd[1]
        tau = float(dd[2]) if len(dd) > 2 else 0.0
        wl = np.exp(-(beta - tau) * e)       # left  factor e^{-(beta - tau) E_m}
        wr = np.exp(-tau * e)                # right factor e^{-tau E_n}
        acc = 0.0
        for i in range(N):
            x, y = i % Lx, i // Lx
            j = ((y + ry) % Ly) * Lx + (x + rx) % Lx
            acc += float(wl @ (X[j] * X[i].T) @ wr) / Z
        out.append(acc / N)
    return np.array(out)


OPS = {"Q": 0, "b": 1, "bd": 2}      # b + b^+, b (annihilation), b^+ (creation)


def correlator_dense(Lx, Ly, beta, t, V, mu, eta, points):
    """Imaginary-time ordered n-point function of H_eta,

        (1/N) sum_i < T prod_k O_k(i + r_k, tau_k) >,

    for points (rx, ry, tau, op) with op in OPS (a name or its code) and tau
    in [0, beta]: the points are ordered by decreasing tau (equal times keep
    their listed order, the first to the left) and the trace is
    Tr(e^{-(beta - tau_1) H} O_1 e^{-(tau_1 - tau_2) H} O_2 ... O_n
    e^{-tau_n H}) / Z."""
    N = Lx * Ly
    H, _, _, _, _ = hamiltonian_dense(Lx, Ly, t, V, mu, eta)
    evals, evecs = np.linalg.eigh(H)
    e = evals - evals.min()
    Z = np.exp(-beta * e).sum()
    states = np.arange(1 << N, dtype=np.int64)

    def op_matrix(code, i):
        code = OPS.get(code, code)
        m = np.zeros((1 << N, 1 << N))
        occ = (states >> i) & 1
        if code in (0, 1):                   # b: |..1_i..> -> |..0_i..>
            src = states[occ == 1]
            m[src ^ (1 << i), src] = 1.0
        if code in (0, 2):                   # b^+: |..0_i..> -> |..1_i..>
            src = states[occ == 0]
            m[src ^ (1 << i), src] = 1.0
        return evecs.T @ m @ evecs

    cache = {}
    order = sorted(range(len(points)), key=lambda k: (-float(points[k][2]), k))
    taus = [float(points[k][2]) for k in order]
    acc = 0.0
    for i in range(N):
        x, y = i % Lx, i // Lx
        prod = np.diag(np.exp(-(beta - taus[0]) * e))
        for n, k in enumerate(order):
            rx, ry, _, op = points[k]
            j = ((y + ry) % Ly) * Lx + (x + rx) % Lx
            key = (OPS.get(op, op), j)
            if key not in cache:
                cache[key] = op_matrix(op, j)
            prod = prod @ cache[key]
            dtau = taus[n] - (taus[n + 1] if n + 1 < len(order) else 0.0)
            prod = prod * np.exp(-dtau * e)[None, :]
        acc += float(np.trace(prod)) / Z
    return acc / N


def _finish(r, N, V, mu, eta):
    E_eta = r["E_eta_total"] / N
    Q = r["Q"] / N
    return {"E": E_eta + eta * Q, "E_eta": E_eta, "n": r["n"] / N, "Q": Q,
            "nn": r["nn"] / N, "K": r["K"] / N}


# --------------------------------------------------------------------------
# translation sectors
# --------------------------------------------------------------------------
def _translate(states, Lx, Ly, dx, dy):
    N = Lx * Ly
    out = np.zeros_like(states)
    for y in range(Ly):
        for x in range(Lx):
            src = y * Lx + x
            dst = ((y + dy) % Ly) * Lx + (x + dx) % Lx
            out |= ((states >> src) & 1) << dst
    return out


def thermal_sectors(Lx, Ly, beta, t, V, mu, eta, verbose=False):
    N = Lx * Ly
    dim = 1 << N
    states = np.arange(dim, dtype=np.int64)
    G = [(dx, dy) for dy in range(Ly) for dx in range(Lx)]
    images = np.stack([_translate(states, Lx, Ly, dx, dy) for dx, dy in G])  # [g, s]
    rep = images.min(axis=0)
    # translation g_s with T^{g_s} rep(s) = s
    img_of_rep = images[:, rep]                       # [g, s] = T^g rep(s)
    gidx = np.argmax(img_of_rep == states[None, :], axis=0)
    stab = (images == states[None, :]).sum(axis=0)    # |S_s|
    reps = np.unique(rep)
    nsum, nn = _diag_parts(Lx, Ly, states)
    gx = np.array([g[0] for g in G])[gidx]
    gy = np.array([g[1] for g in G])[gidx]

    # off-diagonal terms on representatives: hops (amplitude -t), flips (-eta)
    bonds = lattice_bonds(Lx, Ly)
    src_l, dst_l, amp_l, q_l = [], [], [], []
    for a, c in bonds:
        m = ((reps >> a) & 1) != ((reps >> c) & 1)
        src_l.append(reps[m]); dst_l.append(reps[m] ^ ((1 << a) | (1 << c)))
        amp_l.append(np.full(m.sum(), -t)); q_l.append(np.zeros(m.sum()))
    for i in range(N):
        src_l.append(reps); dst_l.append(reps ^ (1 << i))
        amp_l.append(np.full(len(reps), -eta)); q_l.append(np.ones(len(reps)))
    src = np.concatenate(src_l); dst = np.concatenate(dst_l)
    amp = np.concatenate(amp_l); qq = np.concatenate(q_l)
    rdst = rep[dst]

    tot = {"n": 0.0, "nn": 0.0, "Q": 0.0, "K": 0.0, "E_eta_total": 0.0}
    Zs = []
    parts = []
    for kx in range(Lx):
        for ky in range(Ly):
            k = (2 * np.pi * kx / Lx, 2 * np.pi * ky / Ly)
            # compatible representatives: exp(i k.g) = 1 on the stabiliser
            ok = np.ones(len(reps), bool)
            for gi, (dx, dy) in enumerate(G):
                fixed = images[gi, reps] == reps
                ph = np.exp(1j * (k[0] * dx + k[1] * dy))
                ok &= ~fixed | np.isclose(ph, 1.0)
            kreps = reps[ok]
            if len(kreps) == 0:
                continue
            pos = -np.ones(dim, np.int64)
            pos[kreps] = np.arange(len(kreps))
            d = len(kreps)
            H = np.zeros((d, d), complex)
            Qm = np.zeros((d, d), complex)
            Km = np.zeros((d, d), complex)
            keep = (pos[src] >= 0) & (pos[rdst] >= 0)
            s_, dd, a_, q_ = src[keep], dst[keep], amp[keep], qq[keep]
            phase = np.exp(1j * (k[0] * gx[dd] + k[1] * gy[dd]))
            fac = np.sqrt(stab[rep[dd]] / stab[s_])
            val = a_ * phase * fac
            I, J = pos[rep[dd]], pos[s_]
            np.add.at(H, (I, J), val)
            qmask = q_ == 1.0
            np.add.at(Qm, (I[qmask], J[qmask]), (phase * fac)[qmask])
            np.add.at(Km, (I[~qmask], J[~qmask]), val[~qmask])
            H[np.arange(d), np.arange(d)] += V * nn[kreps] - mu * nsum[kreps]
            ev, U = np.linalg.eigh(H)
            prob = np.abs(U) ** 2
            dq = np.real(np.einsum("in,in->n", U.conj(), Qm @ U))
            dk = np.real(np.einsum("in,in->n", U.conj(), Km @ U))
            parts.append((ev, nsum[kreps] @ prob, nn[kreps] @ prob, dq, dk))
            if verbose:
                print("sector", kx, ky, d, flush=True)
    emin = min(p[0].min() for p in parts)
    Z = 0.0
    for ev, dn, dnn, dq, dk in parts:
        w = np.exp(-beta * (ev - emin))
        Z += w.sum()
        tot["n"] += (w * dn).sum(); tot["nn"] += (w * dnn).sum()
        tot["Q"] += (w * dq).sum(); tot["K"] += (w * dk).sum()
        tot["E_eta_total"] += (w * ev).sum()
    r = {k: float(v / Z) for k, v in tot.items()}
    return _finish(r, N, V, mu, eta)


def single_site(beta, mu, eta):
    """Closed form for t = 0, V = 0: every site is H = -mu n - eta sigma^x."""
    R = np.sqrt(mu * mu / 4 + eta * eta)
    th = np.tanh(beta * R)
    return {"Q": eta / R * th, "n": 0.5 * (1 + mu / (2 * R) * th),
            "E": -mu * 0.5 * (1 + mu / (2 * R) * th)}
