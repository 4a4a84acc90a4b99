"""Seeded synthetic workloads (shared by the library tests, the benchmark and the oracle).

This module only builds inputs: mesh descriptions, material constants, and
nodal fields (initial cracks, displacement iterates, constraint bits,
direction vectors) in the library's vector layout.  It contains none of the
solver's arithmetic.  Seeds use numpy.random.default_rng(seed).

Vector layout: component-major blocks [u_1 | ... | u_d | phi], each over the
bounding-box node lattice of the level (Q_p: p*N+1 nodes per axis), x fastest.

Initial cracks follow the AT2 optimal profile phi = 1 - exp(-dist/eps) at the
nodes, dist = Euclidean distance to the crack set; phi^old = phi~ = phi_0.
eps is given in multiples of the element diameter h (the paper's
multiple-fracture setting states eps relative to the element diameter).
"""
from __future__ import annotations

import math

import numpy as np

BOX, LSHAPE = 0, 1
ALL_FACES_2D = 0b1111
ALL_FACES_3D = 0b111111


def spec(name, dim, degree, n, n_levels, domain=BOX, faces=None, E=1.0, nu=0.3, G_c=1.0,
         eps_h=2.0, kappa=1e-10, pressure=1e-3, cracks=(), vcycle="f64", u_amp=0.0, u_seed=0,
         active_target=None, band_eta=1e-2, off_eta=0.0, strip=None, extent=None):
    if faces is None:
        faces = ALL_FACES_3D if dim == 3 else ALL_FACES_2D
    extent = tuple(extent or (1.0,) * dim)
    h = math.sqrt(sum((e / n) ** 2 for e in extent))
    return dict(name=name, dim=dim, degree=degree, n_cells=(n,) * dim, extent=extent,
                n_levels=n_levels, domain=domain, faces=faces,
                material=dict(E=E, nu=nu, G_c=G_c, eps=eps_h * h, kappa=kappa, pressure=pressure),
                h=h, cracks=list(cracks), vcycle=vcycle, u_amp=u_amp, u_seed=u_seed,
                active_target=active_target, band_eta=band_eta, off_eta=off_eta, strip=strip)


def config(name):
    """The named workloads (sizes of the paper's test families, synthetic data).

    A name ending in "_miehe" is the named workload with the Miehe spectral split
    (Sec. 2.1) in place of the unsplit energy: material["split"] = "miehe".
    """
    if name.endswith("_miehe"):
        s = config(name[: -len("_miehe")])
        s["name"] = name
        s["material"] = dict(s["material"], split="miehe")
        return s
    if name == "cfg1_2d_q1_32":
        # 2D unit square 32^2 Q1, crack segment of length 0.25 at the centre, 3 levels
        return spec(name, 2, 1, 32, 3, cracks=[("segment", (0.375, 0.5), (0.625, 0.5))])
    if name == "cfg2_3d_q1_64":
        # 3D unit cube 64^3 Q1, penny crack radius 0.2, 5 levels, plain FP64 V-cycle
        return spec(name, 3, 1, 64, 5, cracks=[("disc", (0.5, 0.5, 0.5), 0.2)],
                    u_amp=1e-3, u_seed=2)
    if name == "cfg3_3d_q2_96":
        # 3D unit cube 96^3 Q2, two penny cracks, ~3% active, FP32 V-cycle
        return spec(name, 3, 2, 96, 5, cracks=[("disc", (0.35, 0.5, 0.4), 0.15),
                                               ("disc", (0.65, 0.5, 0.6), 0.15)],
                    u_amp=1e-3, u_seed=3, vcycle="f32", active_target=0.03, off_eta=0.05)
    if name == "cfg5_3d_q1_lshape_256":
        # L-shaped panel on a 256^3 lattice, 6 levels, damage strip from the re-entrant edge
        return spec(name, 3, 1, 256, 6, domain=LSHAPE, faces=1 << 2, pressure=0.0,
                    cracks=[("strip", 0.5, (0.25, 0.5))], vcycle="f32", active_target=0.05, off_eta=0.02,
                    strip=dict(x=0.5, y_min=0.94, comp=0, value=1e-3))
    if name == "r1_2d_q1_4096":
        return spec(name, 2, 1, 4096, 8, cracks=[("segment", (0.375, 0.5), (0.625, 0.5))])
    # small variants used by parity tests
    if name == "tiny2d":
        return spec(name, 2, 1, 4, 2, cracks=[("segment", (0.25, 0.5), (0.75, 0.5))], u_amp=1e-2, u_seed=7)
    if name == "tiny2d_q2":
        return spec(name, 2, 2, 4, 2, cracks=[("segment", (0.25, 0.5), (0.75, 0.5))], u_amp=1e-2, u_seed=8)
    if name == "tiny3d":
        return spec(name, 3, 1, 4, 2, cracks=[("disc", (0.5, 0.5, 0.5), 0.3)], u_amp=1e-2, u_seed=9)
    if name == "tiny3d_q2":
        return spec(name, 3, 2, 4, 2, cracks=[("disc", (0.5, 0.5, 0.5), 0.3)], u_amp=1e-2, u_seed=10)
    if name == "small2d":
        return spec(name, 2, 1, 24, 3, cracks=[("segment", (0.3, 0.45), (0.7, 0.55))], u_amp=1e-3, u_seed=11)
    if name == "small3d":
        return spec(name, 3, 1, 12, 3, cracks=[("disc", (0.5, 0.5, 0.5), 0.25)], u_amp=1e-3, u_seed=12)
    if name == "small3d_q2":
        return spec(name, 3, 2, 8, 3, cracks=[("disc", (0.5, 0.5, 0.5), 0.25)], u_amp=1e-3, u_seed=13,
                    vcycle="f32", active_target=0.03, off_eta=0.05)
    if name == "small_lshape":
        return spec(name, 3, 1, 16, 3, domain=LSHAPE, faces=1 << 2, pressure=0.0,
                    cracks=[("strip", 0.5, (0.25, 0.5))], vcycle="f32", active_target=0.05, off_eta=0.02,
                    strip=dict(x=0.5, y_min=0.94, comp=0, value=1e-3))
    if name == "mid_lshape":
        return spec(name, 3, 1, 64, 4, domain=LSHAPE, faces=1 << 2, pressure=0.0,
                    cracks=[("strip", 0.5, (0.25, 0.5))], vcycle="f32", active_target=0.05, off_eta=0.02,
                    strip=dict(x=0.5, y_min=0.94, comp=0, value=1e-3))
    if name == "mid3d_q2":
        return spec(name, 3, 2, 24, 3, cracks=[("disc", (0.35, 0.5, 0.4), 0.15),
                                               ("disc", (0.65, 0.5, 0.6), 0.15)],
                    u_amp=1e-3, u_seed=3, vcycle="f32", active_target=0.03, off_eta=0.05)
    raise KeyError(name)


NAMES = ["cfg1_2d_q1_32", "cfg2_3d_q1_64", "cfg3_3d_q2_96", "cfg5_3d_q1_lshape_256"]


def scaled(s, n, n_levels):
    """The same recipe on n cells per axis (a scaled-down replica): eps keeps its multiple of
    the element diameter, every other parameter is unchanged."""
    h = math.sqrt(sum((e / n) ** 2 for e in s["extent"]))
    out = dict(s, n_cells=(n,) * s["dim"], n_levels=n_levels, h=h, name=f"{s['name']}@{n}")
    out["material"] = dict(s["material"], eps=s["material"]["eps"] / s["h"] * h)
    return out


# --------------------------------------------------------------------------
# geometry of the node lattice
# --------------------------------------------------------------------------
def lattice(s, level_from_top=0):
    """Node counts per axis and node coordinates (n_nodes, d) on a level (0 = finest)."""
    d, p = s["dim"], s["degree"]
    N = [n >> level_from_top for n in s["n_cells"]]
    nn = [p * n + 1 for n in N]
    axes = [np.arange(m) * (e / (m - 1)) for m, e in zip(nn, s["extent"])]
    grids = np.meshgrid(*axes[::-1], indexing="ij")
    X = np.stack([g.ravel() for g in grids[::-1]], axis=1)
    return nn, X


def hole_nodes(s, X):
    if s["domain"] != LSHAPE:
        return np.zeros(X.shape[0], dtype=bool)
    ex, ey = s["extent"][0], s["extent"][1]
    return (X[:, 0] > 0.5 * ex + 1e-12) & (X[:, 1] > 0.5 * ey + 1e-12)


def face_nodes(s, X):
    sel = np.zeros(X.shape[0], dtype=bool)
    for k in range(s["dim"]):
        if s["faces"] & (1 << (2 * k)):
            sel |= np.abs(X[:, k]) < 1e-12
        if s["faces"] & (1 << (2 * k + 1)):
            sel |= np.abs(X[:, k] - s["extent"][k]) < 1e-12
    return sel


def crack_distance(s, X):
    dist = np.full(X.shape[0], np.inf)
    for c in s["cracks"]:
        kind = c[0]
        if kind == "segment":
            a, b = np.array(c[1]), np.array(c[2])
            ab = b - a
            t = np.clip(((X - a) @ ab) / (ab @ ab), 0.0, 1.0)
            dd = np.linalg.norm(X - (a + t[:, None] * ab), axis=1)
        elif kind == "disc":
            ctr, r = np.array(c[1]), c[2]
            rho = np.hypot(X[:, 0] - ctr[0], X[:, 1] - ctr[1])
            dd = np.hypot(X[:, 2] - ctr[2], np.maximum(0.0, rho - r))
        elif kind == "strip":
            y0, (x0, x1) = c[1], c[2]
            dx = np.maximum(0.0, np.maximum(x0 - X[:, 0], X[:, 0] - x1))
            dd = np.hypot(X[:, 1] - y0, dx)
        else:
            raise ValueError(kind)
        dist = np.minimum(dist, dd)
    return dist


def strip_nodes(s, X):
    st = s.get("strip")
    if not st:
        return np.zeros(X.shape[0], dtype=bool)
    return (np.abs(X[:, 0] - st["x"]) < 1e-12) & (X[:, 1] >= st["y_min"] - 1e-12)


def extra_constraint_bits(s):
    """Per-node bits (bit i = displacement component i) of the prescribed-displacement strip, or None."""
    st = s.get("strip")
    if not st:
        return None
    _, X = lattice(s)
    bits = np.zeros(X.shape[0], dtype=np.uint8)
    bits[strip_nodes(s, X)] |= np.uint8(1 << st["comp"])
    return bits


# --------------------------------------------------------------------------
# fields
# --------------------------------------------------------------------------
def make_state(s):
    """(U_k, U_old, phi~) on the finest level for one Newton step of the workload.

    u_k: seeded uniform(-u_amp, u_amp) on displacement DoFs off the Dirichlet
    faces and the hole (zero there), plus the prescribed strip value.
    phi^old = phi~ = 1 - exp(-dist/eps); hole nodes are zero in every component.
    With an active-set target fraction, the iterate sits in the middle of the
    active-set loop: phi_k = min(1, phi^old + band_eta) on the band dist <= d*
    holding that fraction of the phase-field nodes (infeasible there, so the
    rule of Algorithm 1 activates it), and phi_k = max(0, phi^old - off_eta)
    elsewhere (feasible, below the constraint, so the rule leaves it free where
    c (phi_k - phi^old) outweighs M^-1 R).  Without the downward shift the
    exp(-d/eps) profile, an equilibrium only in 1D, activates most phi-nodes
    around curved crack fronts and boundaries.  off_eta = 0.02 (L-panel) and
    0.05 (two penny cracks, Q2) put 5.1% and 3.0% of the phi-nodes in the
    active set of the 256^3 and 96^3 meshes.
    """
    d = s["dim"]
    _, X = lattice(s)
    nn = X.shape[0]
    hole = hole_nodes(s, X)
    eps = s["material"]["eps"]
    dist = crack_distance(s, X)
    phi_old = 1.0 - np.exp(-dist / eps)
    phi_old[hole] = 0.0
    U = np.zeros((d + 1) * nn)
    if s["u_amp"] > 0:
        rng = np.random.default_rng(s["u_seed"])
        u = rng.uniform(-s["u_amp"], s["u_amp"], size=d * nn)
        fixed = face_nodes(s, X) | hole
        for i in range(d):
            u[i * nn:(i + 1) * nn][fixed] = 0.0
        U[:d * nn] = u
    st = s.get("strip")
    if st:
        sn = strip_nodes(s, X)
        U[st["comp"] * nn:(st["comp"] + 1) * nn][sn] = st["value"]
    phi = phi_old.copy()
    if s.get("active_target"):
        live = ~hole
        k = int(round(s["active_target"] * live.sum()))
        dstar = np.sort(dist[live])[max(k - 1, 0)]
        band = live & (dist <= dstar)
        phi[band] = np.minimum(1.0, phi_old[band] + s["band_eta"])
        off = live & ~band
        phi[off] = np.maximum(0.0, phi_old[off] - s.get("off_eta", 0.0))
    U[d * nn:] = phi
    U_old = U.copy()
    U_old[d * nn:] = phi_old
    return U, U_old, phi_old.copy()


def random_linearization(s, seed, u_amp=1e-3):
    """A generic linearization point: u ~ U(-u_amp, u_amp), phi ~ U(0, 1), phi~ ~ U(0, 1) (hole = 0)."""
    d = s["dim"]
    _, X = lattice(s)
    nn = X.shape[0]
    hole = hole_nodes(s, X)
    rng = np.random.default_rng(seed)
    U = np.concatenate([rng.uniform(-u_amp, u_amp, d * nn), rng.uniform(0.0, 1.0, nn)])
    phit = rng.uniform(0.0, 1.0, nn)
    for c in range(d + 1):
        U[c * nn:(c + 1) * nn][hole] = 0.0
    phit[hole] = 0.0
    return U, phit


def random_vector(s, seed, level_from_top=0):
    """x ~ U(-1, 1) on every DoF of a level (the apply's direction vector)."""
    nn, _ = lattice(s, level_from_top)
    n = (s["dim"] + 1) * int(np.prod(nn))
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def random_active(s, seed, frac=0.1):
    """A seeded random 0/1 active indicator on the finest-level nodes (hole excluded)."""
    _, X = lattice(s)
    hole = hole_nodes(s, X)
    a = np.random.default_rng(seed).uniform(size=X.shape[0]) < frac
    return (a & ~hole).astype(np.uint8)


def batched_instances(seed=4, count=64):
    """The batched 2D family: log-uniform mesh sizes 16..256 (multiples of 8), 4 levels each,
    eps ~ U(h, 4h), pressure log-uniform in [1e-4, 1e-2], 1-3 random straight cracks."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(8 * round(math.exp(rng.uniform(math.log(16), math.log(256))) / 8))
        h = math.sqrt(2.0) / n
        eps_h = rng.uniform(1.0, 4.0)
        pres = math.exp(rng.uniform(math.log(1e-4), math.log(1e-2)))
        k = int(rng.integers(1, 4))
        cracks = []
        for _ in range(k):
            c = rng.uniform(0.25, 0.75, 2)
            ang = rng.uniform(0.0, math.pi)
            ln = rng.uniform(0.1, 0.3)
            dv = 0.5 * ln * np.array([math.cos(ang), math.sin(ang)])
            cracks.append(("segment", tuple(c - dv), tuple(c + dv)))
        out.append(spec(f"batch{i}", 2, 1, n, 4, eps_h=eps_h, pressure=pres, cracks=cracks,
                        vcycle="f32"))
        assert abs(out[-1]["h"] - h) < 1e-15
    return out
