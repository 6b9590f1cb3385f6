"""Seeded generators for particle configurations, forces and kernel weights.

Every random number comes from numpy's PCG64 bit generator as raw 64-bit words
(a stream that numpy keeps stable across versions) and is mapped to uniforms
and normals here, so the values do not depend on numpy's distribution code.

Workload recipes follow the paper's synthetic set-ups: spheres of radius a=1 in
an unbounded fluid (Sec. 2.1), perturbed primitive cubic lattices (Sec. 4.1),
spherical suspension drops built as lattice points inside a ball and then
jittered, under gravity-like forces F=(0,0,-1) (Sec. 4.3.1), and bead chains
for flexible filaments (Sec. 4.3.2).
"""
from __future__ import annotations

import math
import os

import numpy as np
from scipy.spatial import cKDTree

_STREAMS = {"pos": 0, "force": 1, "weights": 2, "rows": 3, "fd": 4, "sizes": 5,
            "kinds": 6, "phi": 7, "chain": 8, "w": 9, "misc": 10}


class Rng:
    """Counter-free wrapper around PCG64 raw output with explicit mappings."""

    def __init__(self, seed: int, stream: str | int = 0):
        sid = _STREAMS[stream] if isinstance(stream, str) else int(stream)
        ss = np.random.SeedSequence([int(seed), sid])
        self._bg = np.random.PCG64(ss)

    def raw(self, n: int) -> np.ndarray:
        return self._bg.random_raw(int(n)).astype(np.uint64)

    def uniform(self, n: int) -> np.ndarray:
        """Doubles in [0, 1) with 53 random bits each."""
        return (self.raw(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def uniform_pm(self, n: int, half: float) -> np.ndarray:
        return (2.0 * self.uniform(n) - 1.0) * half

    def normal(self, n: int) -> np.ndarray:
        """Standard normals by the Box-Muller transform (pairs of uniforms)."""
        m = (int(n) + 1) // 2
        u1 = 1.0 - self.uniform(m)          # (0, 1]
        u2 = self.uniform(m)
        rad = np.sqrt(-2.0 * np.log(u1))
        z = np.empty(2 * m)
        z[0::2] = rad * np.cos(2.0 * np.pi * u2)
        z[1::2] = rad * np.sin(2.0 * np.pi * u2)
        return z[: int(n)]


def cube_side(n: int, phi: float, a: float = 1.0) -> float:
    """Side of the cube holding n spheres of radius a at volume fraction phi."""
    return a * (4.0 * math.pi * n / (3.0 * phi)) ** (1.0 / 3.0)


def drop_radius(n: int, phi: float, a: float = 1.0) -> float:
    return a * (n / phi) ** (1.0 / 3.0)


def _cached(name, fn):
    """Memoise a generated array in a local directory (inputs are deterministic)."""
    d = os.environ.get("HH_INPUT_CACHE", "/tmp/hh_inputs")
    path = os.path.join(d, name + ".npy")
    try:
        return np.load(path)
    except (OSError, ValueError):
        pass
    arr = fn()
    try:
        os.makedirs(d, exist_ok=True)
        tmp = path + ".%d.tmp" % os.getpid()
        with open(tmp, "wb") as f:
            np.save(f, arr)
        os.replace(tmp, path)
    except OSError:
        pass
    return arr


def rsa_cube(n: int, phi: float, min_dist: float = 2.05, a: float = 1.0,
             seed: int = 0, batch: int = 4096) -> np.ndarray:
    """Cached front end of _rsa_cube (see there)."""
    key = "rsa_n%d_phi%.6g_d%.6g_a%.6g_s%d_b%d" % (n, phi, min_dist, a, seed, batch)
    if n < 20000:
        return _rsa_cube(n, phi, min_dist, a, seed, batch)
    return _cached(key, lambda: _rsa_cube(n, phi, min_dist, a, seed, batch))


def _rsa_cube(n: int, phi: float, min_dist: float = 2.05, a: float = 1.0,
              seed: int = 0, batch: int = 4096) -> np.ndarray:
    """Random sequential addition of n centres uniform in [0, L)^3.

    A candidate is accepted when its distance to every earlier accepted centre
    is at least min_dist. Candidates are drawn in batches, but the acceptance
    decision is exactly the sequential one in draw order.
    """
    n = int(n)
    L = cube_side(n, phi, a)
    rng = Rng(seed, "pos")
    nc = max(1, int(math.floor(L / min_dist)))
    w = L / nc
    slots = 8
    grid = np.full((nc, nc, nc, slots), -1, dtype=np.int64)
    fill = np.zeros((nc, nc, nc), dtype=np.int64)
    pos = np.empty((n, 3))
    count = 0
    d2min = min_dist * min_dist
    offs = np.array([(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)])
    tries = 0
    while count < n:
        tries += 1
        if tries > 100000:
            raise RuntimeError("rsa_cube: volume fraction too high to place spheres")
        cand = rng.uniform(3 * batch).reshape(batch, 3) * L
        cell = np.minimum((cand / w).astype(np.int64), nc - 1)
        nb = cell[:, None, :] + offs[None, :, :]                       # [B,27,3]
        ok_cell = np.all((nb >= 0) & (nb < nc), axis=2)
        nbc = np.clip(nb, 0, nc - 1)
        idx = grid[nbc[..., 0], nbc[..., 1], nbc[..., 2]]              # [B,27,slots]
        idx = np.where(ok_cell[..., None], idx, -1).reshape(batch, -1)
        valid = idx >= 0
        p = pos[np.where(valid, idx, 0)]
        d2 = np.sum((p - cand[:, None, :]) ** 2, axis=2)
        clash = np.any(valid & (d2 < d2min), axis=1)
        surv = np.nonzero(~clash)[0]
        if surv.size:
            cs = cand[surv]
            pairs = cKDTree(cs).query_pairs(min_dist, output_type="ndarray")
            if pairs.size:   # drop pairs at exactly min_dist (allowed)
                dp = cs[pairs[:, 0]] - cs[pairs[:, 1]]
                pairs = pairs[np.sum(dp * dp, axis=1) < d2min]
            acc_mask = np.ones(surv.size, dtype=bool)
            if pairs.size:
                # only candidates that clash with another batch member need the
                # sequential rule: accepted iff no earlier accepted member clashes
                earlier = {}
                for u, v in pairs.tolist():
                    lo_, hi_ = (u, v) if u < v else (v, u)
                    earlier.setdefault(hi_, []).append(lo_)
                for t in sorted(set(earlier) | {u for lst in earlier.values() for u in lst}):
                    acc_mask[t] = not any(acc_mask[u] for u in earlier.get(t, ()))
            accepted = np.nonzero(acc_mask)[0][: n - count]
            for t in accepted:
                c = cell[surv[t]]
                f = fill[c[0], c[1], c[2]]
                if f >= slots:
                    raise RuntimeError("rsa_cube: cell overflow")
                grid[c[0], c[1], c[2], f] = count
                fill[c[0], c[1], c[2]] = f + 1
                pos[count] = cs[t]
                count += 1
    return pos


def lattice_sphere(n: int, phi: float, jitter: float = 0.25, a: float = 1.0,
                   seed: int = 0) -> np.ndarray:
    """n points of a primitive cubic lattice nearest the centre, then jittered.

    Lattice spacing s = a (4 pi / (3 phi))^(1/3) gives volume fraction phi.
    Points are ranked by squared integer distance from the centre with a
    lexicographic tie-break, and each coordinate is then moved by U(-jitter a,
    jitter a), which keeps centres at least s - 2 sqrt(3) jitter a apart.
    """
    n = int(n)
    s = a * (4.0 * math.pi / (3.0 * phi)) ** (1.0 / 3.0)
    m = int(math.ceil((3.0 * n / (4.0 * math.pi)) ** (1.0 / 3.0))) + 2
    r = np.arange(-m, m + 1, dtype=np.int64)
    I, J, K = np.meshgrid(r, r, r, indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    d2 = I * I + J * J + K * K
    order = np.lexsort((K, J, I, d2))[:n]
    pts = np.stack([I[order], J[order], K[order]], axis=1).astype(np.float64) * s
    del I, J, K, d2, order
    rng = Rng(seed, "pos")
    pts += rng.uniform_pm(3 * n, jitter * a).reshape(n, 3)
    return pts


def lattice_cube(n: int, phi: float, jitter: float = 0.25, a: float = 1.0,
                 seed: int = 0) -> np.ndarray:
    """n points of a primitive cubic lattice filling a cube row by row (the
    paper's perturbed-lattice construction, Sec. 4.1), jittered by U(+-j a) with
    j = min(jitter, (s - 2.05 a) / (2 sqrt(3) a)) so centres stay >= 2.05 a apart."""
    n = int(n)
    s = a * (4.0 * math.pi / (3.0 * phi)) ** (1.0 / 3.0)
    jitter = max(0.0, min(jitter, (s - 2.05 * a) / (2.0 * math.sqrt(3.0) * a)))
    m = int(math.ceil(n ** (1.0 / 3.0)))
    i = np.arange(n, dtype=np.int64)
    pts = np.stack([i % m, (i // m) % m, i // (m * m)], axis=1).astype(np.float64) * s
    rng = Rng(seed, "pos")
    pts += rng.uniform_pm(3 * n, jitter * a).reshape(n, 3)
    return pts


def filament_chains(n: int, phi: float, beads: int = 50, bond: float = 2.2,
                    bend_sd: float = 0.3, a: float = 1.0, seed: int = 0) -> np.ndarray:
    """Chains of `beads` beads (n rounded down to a multiple of beads).

    Chain starts are uniform in the cube sized for phi; each bond has length
    `bond` and turns from the previous bond by a polar angle |theta|, theta ~
    N(0, bend_sd), with uniform azimuth. Beads of different chains are not
    kept apart (no overlap resolution across chains).
    """
    nchain = max(1, int(n) // beads)
    L = cube_side(nchain * beads, phi, a)
    rng = Rng(seed, "chain")
    pos = np.empty((nchain, beads, 3))
    pos[:, 0] = rng.uniform(3 * nchain).reshape(nchain, 3) * L
    d = rng.normal(3 * nchain).reshape(nchain, 3)
    d /= np.linalg.norm(d, axis=1)[:, None]
    for b in range(1, beads):
        th = np.abs(rng.normal(nchain)) * bend_sd
        ps = rng.uniform(nchain) * 2.0 * math.pi
        hp = np.where(np.abs(d[:, :1]) < 0.9, [[1.0, 0.0, 0.0]], [[0.0, 1.0, 0.0]])
        u = np.cross(d, hp)
        u /= np.linalg.norm(u, axis=1)[:, None]
        v = np.cross(d, u)
        d = (np.cos(th)[:, None] * d + np.sin(th)[:, None] *
             (np.cos(ps)[:, None] * u + np.sin(ps)[:, None] * v))
        pos[:, b] = pos[:, b - 1] + bond * a * d
    return pos.reshape(-1, 3)


def filament_suspension(n_fil: int = 5120, n_beads: int = 21, bond: float = 3.0,
                        n_free: int = 107520, min_dist: float = 2.1, seed: int = 0):
    """A spherical cloud of straight filaments and free particles, the shape of
    the flexible-filament workload of Sec. 4.3.2: outer radius
    R_out = 4 * 10^(1/3) * (n_beads - 1) * bond; the filaments (n_beads beads
    at spacing `bond`, random orientation) lie inside R_in = (1/2)^(1/3) R_out,
    the free particles uniformly in the shell between R_in and R_out; no two
    particles closer than min_dist (a candidate that clashes is drawn again).
    Returns X with the filaments first (chain c = particles
    [c n_beads, (c + 1) n_beads)), then the free particles."""
    key = "filsusp_f%d_b%d_l%.6g_p%d_d%.6g_s%d" % (n_fil, n_beads, bond, n_free, min_dist, seed)
    return _cached(key, lambda: _filament_suspension(n_fil, n_beads, bond, n_free, min_dist,
                                                     seed))


def _filament_suspension(n_fil, n_beads, bond, n_free, min_dist, seed):
    r_out = 4.0 * 10.0 ** (1.0 / 3.0) * (n_beads - 1) * bond
    r_in = 0.5 ** (1.0 / 3.0) * r_out
    half = 0.5 * (n_beads - 1) * bond
    rng = Rng(seed, "chain")
    offs = (np.arange(n_beads) - 0.5 * (n_beads - 1)) * bond
    placed = np.empty((0, 3))
    chains = []
    while len(chains) < n_fil:
        m = n_fil - len(chains)
        # centres uniform in the ball of radius r_in - half (so every bead is
        # inside r_in), by rejection from the cube; directions uniform
        c = (rng.uniform(3 * 2 * m).reshape(2 * m, 3) * 2.0 - 1.0) * (r_in - half)
        c = c[np.sum(c * c, axis=1) <= (r_in - half) ** 2][:m]
        d = rng.normal(3 * c.shape[0]).reshape(-1, 3)
        d /= np.linalg.norm(d, axis=1)[:, None]
        beads = c[:, None, :] + offs[None, :, None] * d[:, None, :]        # [m, nb, 3]
        ok = np.ones(c.shape[0], dtype=bool)
        if placed.shape[0]:
            dist, _ = cKDTree(placed).query(beads.reshape(-1, 3), k=1)
            ok &= ~np.any(dist.reshape(-1, n_beads) < min_dist, axis=1)
        flat = beads.reshape(-1, 3)
        pairs = cKDTree(flat).query_pairs(min_dist, output_type="ndarray")
        for u, v in pairs.tolist():
            cu, cv = u // n_beads, v // n_beads
            if cu != cv and ok[min(cu, cv)]:
                ok[max(cu, cv)] = False     # the later chain of a clashing pair is redrawn
        for t in np.nonzero(ok)[0]:
            chains.append(beads[t])
        placed = np.concatenate([placed, beads[ok].reshape(-1, 3)])
    rng2 = Rng(seed, "pos")
    free = np.empty((0, 3))
    while free.shape[0] < n_free:
        m = 2 * (n_free - free.shape[0]) + 64
        p = (rng2.uniform(3 * m).reshape(m, 3) * 2.0 - 1.0) * r_out
        rr = np.sum(p * p, axis=1)
        p = p[(rr <= r_out * r_out) & (rr >= r_in * r_in)]
        allp = np.concatenate([placed, free])
        dist, _ = cKDTree(allp).query(p, k=1)
        p = p[dist >= min_dist]
        keep = np.ones(p.shape[0], dtype=bool)
        for u, v in cKDTree(p).query_pairs(min_dist, output_type="ndarray").tolist():
            if keep[min(u, v)]:
                keep[max(u, v)] = False
        free = np.concatenate([free, p[keep]])[:n_free]
    return np.concatenate([np.concatenate(chains)[: n_fil * n_beads], free])


def normal_forces(n: int, seed: int = 0, scale: float = 1.0,
                  dtype=np.float64) -> np.ndarray:
    """F_i ~ N(0, scale^2 I3)."""
    rng = Rng(seed, "force")
    return (scale * rng.normal(3 * int(n)).reshape(int(n), 3)).astype(dtype)


def gravity_forces(n: int, seed: int = 0, var: float = 0.1,
                   dtype=np.float64) -> np.ndarray:
    """F_i = (0, 0, -1) + N(0, var I3)."""
    f = normal_forces(n, seed, math.sqrt(var))
    f[:, 2] -= 1.0
    return f.astype(dtype)


def mlp_weights(seed: int = 1, widths=(3, 64, 64, 64, 9)):
    """Glorot-uniform weights W[out][in] ~ U(+-sqrt(6/(in+out))), biases
    b ~ U(+-1/sqrt(in)), drawn in the order W1, b1, W2, b2, ... from one stream."""
    rng = Rng(seed, "weights")
    Ws, bs = [], []
    for fin, fout in zip(widths[:-1], widths[1:]):
        lim = math.sqrt(6.0 / (fin + fout))
        Ws.append(rng.uniform_pm(fout * fin, lim).reshape(fout, fin))
        bs.append(rng.uniform_pm(fout, 1.0 / math.sqrt(fin)))
    return Ws, bs


def sample_rows(n: int, k: int, seed: int = 3) -> np.ndarray:
    """k distinct row indices of [0, n), uniform without replacement, ascending."""
    rng = Rng(seed, "rows")
    keys = rng.raw(int(n))
    pick = np.argsort(keys, kind="stable")[: int(k)]
    return np.sort(pick).astype(np.int64)


def batch_systems(n_sys: int = 64, nmin: int = 5000, nmax: int = 200000, seed: int = 2):
    """Per-system sizes (log-uniform in [nmin, nmax]), kinds and volume fractions.

    Even-numbered systems are free spheres, odd-numbered ones are filaments.
    Returns a list of dicts {n, kind, phi, seed}.
    """
    rs = Rng(seed, "sizes")
    u = rs.uniform(n_sys)
    sizes = np.floor(np.exp(math.log(nmin) + u * (math.log(nmax) - math.log(nmin)))).astype(np.int64)
    rp = Rng(seed, "phi")
    phis = 0.05 + 0.25 * rp.uniform(n_sys)
    out = []
    for s in range(n_sys):
        kind = "spheres" if s % 2 == 0 else "filaments"
        n = int(sizes[s])
        if kind == "filaments":
            n = max(50, (n // 50) * 50)
        out.append({"n": n, "kind": kind, "phi": float(phis[s]), "seed": 1000 + s})
    return out


def batch_workload(n_sys: int = 64, nmin: int = 5000, nmax: int = 200000, seed: int = 2):
    """Positions, forces and offsets of the batched workload: even systems are
    free spheres (perturbed lattice in a cube at phi ~ U[0.05, 0.30]), odd ones
    flexible filaments (50-bead chains, bond 2.2 a, bending N(0, 0.3))."""
    specs = batch_systems(n_sys, nmin, nmax, seed)
    Xs, Fs, off = [], [], [0]
    for sp in specs:
        if sp["kind"] == "spheres":
            X = lattice_cube(sp["n"], sp["phi"], seed=sp["seed"])
        else:
            X = filament_chains(sp["n"], sp["phi"], seed=sp["seed"])
        Xs.append(X)
        Fs.append(normal_forces(X.shape[0], seed=sp["seed"]))
        off.append(off[-1] + X.shape[0])
    return np.concatenate(Xs), np.concatenate(Fs), np.asarray(off, dtype=np.int64), specs


# Named workloads (positions generator, forces, kernel, H-matrix parameters).
WORKLOADS = {
    "plain_small": dict(n=2000, geom="cube", phi=0.10, seed=0, forces="normal",
                        kernel="rpy", precision="fp64", c_leaf=64, eta=1.0, eps=1e-6),
    "plain_fp32": dict(n=100000, geom="cube", phi=0.20, seed=0, forces="normal",
                       kernel="mlp", precision="fp32", c_leaf=128, eta=1.0, eps=1e-4),
    "precision_1m": dict(n=1000000, geom="sphere", phi=0.10, seed=0, forces="gravity",
                         kernel="mlp", precision="bf16", c_leaf=128, eta=1.0, eps=1e-4),
    "precision_10m": dict(n=10000000, geom="sphere", phi=0.10, seed=0, forces="gravity",
                          kernel="mlp", precision="bf16", c_leaf=128, eta=1.0, eps=1e-4),
    "diff_200k": dict(n=200000, geom="cube", phi=0.15, seed=0, forces="normal",
                      kernel="mlp", precision="fp32", c_leaf=128, eta=1.0, eps=1e-4),
    "diff_5k": dict(n=5000, geom="cube", phi=0.15, seed=0, forces="normal",
                    kernel="mlp", precision="fp32", c_leaf=128, eta=1.0, eps=1e-4),
    # the flexible-filament suspension (5,120 chains of 21 beads, 107,520 free
    # particles) under gravity with tension and bending, stepped in time
    "filaments_215k": dict(n=215040, geom="filaments", phi=None, seed=0, forces="gravity",
                           kernel="mlp", precision="bf16", c_leaf=128, eta=1.0, eps=0.02,
                           n_fil=5120, n_beads=21, bond=3.0, dt=0.002, k_t=20.0, k_b=50.0),
    # the 6N product with rotations: forces and torques ~ N(0, I3) on 1M
    # particles of the plain random suspension (F holds (F_i, T_i), [n][6])
    "rotation_1m": dict(n=1000000, geom="cube", phi=0.20, seed=0, forces="normal+torques",
                        kernel="rpy6", precision="fp32", c_leaf=64, eta=1.0, eps=1e-5),
    # 64 independent systems (batch_workload): n is the total, set when generated
    "batch64": dict(n=None, geom="batch", phi=None, seed=2, forces="normal",
                    kernel="mlp", precision="bf16", c_leaf=128, eta=1.0, eps=1e-4),
}


def workload(name: str, n: int | None = None):
    """Positions and forces of a named workload (optionally at another n)."""
    w = dict(WORKLOADS[name])
    if w["geom"] == "batch":
        X, F, off, specs = batch_workload(seed=w["seed"])
        w["n"] = int(X.shape[0])
        w["offsets"] = off
        w["systems"] = specs
        return X, F, w
    if n is not None:
        w["n"] = int(n)
    if w["geom"] == "filaments":
        # n (if given) scales both parts, keeping the equal split of Sec. 4.3.2
        nf = max(1, int(round(w["n_fil"] * w["n"] / 215040)))
        X = filament_suspension(nf, w["n_beads"], w["bond"], nf * w["n_beads"], seed=w["seed"])
        w["n_fil"], w["n"] = nf, int(X.shape[0])
        return X, np.tile([0.0, 0.0, -1.0], (X.shape[0], 1)), w
    if w["geom"] == "cube":
        X = rsa_cube(w["n"], w["phi"], seed=w["seed"])
    else:
        X = lattice_sphere(w["n"], w["phi"], seed=w["seed"])
    if w["forces"] == "normal":
        F = normal_forces(w["n"], seed=w["seed"])
    elif w["forces"] == "normal+torques":
        F = np.hstack([normal_forces(w["n"], seed=w["seed"]),
                       normal_forces(w["n"], seed=w["seed"] + 1)])
    else:
        F = gravity_forces(w["n"], seed=w["seed"])
    return X, F, w
