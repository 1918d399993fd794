"""Seeded synthetic workloads for the 2D P1 Helmholtz problems.

Conventions (shared by every consumer):
  * structured N x N node grid on the unit square [0,1]^2, h = 1/(N-1);
  * node (i, j) sits at (i*h, j*h) and has id j*N + i;
  * a source is a Gaussian bump exp(-|x - x0|^2 / (2 w^2)) of amplitude 1,
    sampled at the nodes (the nodal interpolant f_I);
  * the speed field c(x) = 1 + 2*sigmoid(g(x)) with g a random-feature
    Gaussian field of correlation length ell; slowness s = 1/c.

Random draws use numpy's PCG64 with explicit seeds, so every array here is a
pure function of its arguments.
"""
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "node_coords", "source_centers", "gaussian_sources",
    "random_field", "speed_field", "make_problem", "CONFIGS", "make_batch", "BATCHES",
    "receiver_nodes", "batch_grid_sizes", "ElasticProblem", "lame_fields",
    "make_elastic", "ELASTIC", "DGProblem", "dg_node_coords", "make_dg", "DG",
    "IpdgProblem", "make_ipdg", "IPDG_FAMILIES", "IPDG_INV_H",
]


def node_coords(N):
    """(x, y) float64 arrays of length N*N, node id = j*N + i."""
    h = 1.0 / (N - 1)
    i = np.arange(N, dtype=np.float64)
    x = np.tile(i, N) * h
    y = np.repeat(i, N) * h
    return x, y


def source_centers(seed, count, lo=0.25, hi=0.75):
    """count source positions drawn uniformly in [lo, hi]^2 (PCG64(seed))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=(count, 2))


def gaussian_sources(N, centers, width=0.02):
    """Nodal samples of Gaussian bumps: array (N*N, len(centers)), float64."""
    x, y = node_coords(N)
    centers = np.asarray(centers, dtype=np.float64).reshape(-1, 2)
    f = np.empty((N * N, centers.shape[0]), dtype=np.float64)
    for s, (cx, cy) in enumerate(centers):
        f[:, s] = np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * width * width))
    return f


def random_field(N, seed, ell=0.1, n_features=1024, device=None):
    """Random-feature Gaussian field g(x) = sqrt(2/M) sum_m cos(w_m.x + b_m),
    w_m ~ N(0, ell^-2 I), b_m ~ U[0, 2pi); unit variance, correlation ell.
    With a torch device the sum is evaluated there (float64) and a tensor is
    returned; the draws are the same."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.normal(0.0, 1.0 / ell, size=(n_features, 2))
    b = rng.uniform(0.0, 2.0 * np.pi, size=n_features)
    x, y = node_coords(N)
    if device is not None:
        import torch
        t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=device)  # noqa: E731
        xt, yt, wt, bt = t(x), t(y), t(w), t(b)
        g = torch.zeros(N * N, dtype=torch.float64, device=device)
        chunk = 1 << 16
        for s in range(0, N * N, chunk):
            ph = (torch.outer(xt[s:s + chunk], wt[:, 0]) + torch.outer(yt[s:s + chunk], wt[:, 1])
                  + bt)
            g[s:s + chunk] = torch.cos(ph).sum(dim=1)
        return g * np.sqrt(2.0 / n_features)
    g = np.zeros(N * N)
    chunk = 4096
    for s in range(0, N * N, chunk):
        ph = np.outer(x[s:s + chunk], w[:, 0]) + np.outer(y[s:s + chunk], w[:, 1]) + b
        g[s:s + chunk] = np.cos(ph).sum(axis=1)
    return g * np.sqrt(2.0 / n_features)


def speed_field(N, seed, ell=0.1, device=None):
    """c(x) = 1 + 2*sigmoid(g(x)) in (1, 3)."""
    g = random_field(N, seed, ell, device=device)
    if device is not None:
        import torch
        return 1.0 + 2.0 * torch.sigmoid(g)
    return 1.0 + 2.0 / (1.0 + np.exp(-g))


def receiver_nodes(N, seed, count=8):
    """count distinct node ids drawn uniformly without replacement."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(N * N, size=count, replace=False)).astype(np.int64)


def batch_grid_sizes(seed, count, lo=65, hi=513):
    """Uneven grid sizes N_i ~ U{lo..hi}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=count).astype(np.int64)


@dataclass
class Problem:
    """One seeded Helmholtz P1 workload: -lap u - (omega s)^2 u = f on [0,1]^2
    with the first-order absorbing condition on all four sides."""
    name: str
    N: int
    omega: float
    slowness: np.ndarray          # (N*N,) float64 nodal slowness s = 1/c
    f: np.ndarray                 # (N*N, nrhs) float64 nodal source samples
    leaf_dofs: int = 32           # nested-dissection leaf size (DOFs)
    beta: int = 16                # HSS leaf size
    tol: float = 1e-6             # HSS compression tolerance
    h_sw: int = 4                 # switching height
    gmres_m: int = 50
    gmres_tol: float = 1e-8
    factor_dtype: str = "c128"
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.N * self.N

    @property
    def nrhs(self):
        return self.f.shape[1]


def _helmholtz(name, N, omega, seed, nsrc, **kw):
    centers = source_centers(seed, nsrc)
    return Problem(name=name, N=N, omega=float(omega),
                   slowness=np.ones(N * N), f=gaussian_sources(N, centers), **kw)


#: Named workloads.  The first is the small case the oracle runs in seconds;
#: the second is the 263k-DOF, 64-source case the benchmark times.
CONFIGS = {
    "helmholtz_p1_65": dict(N=65, omega=16.0, seed=0, nsrc=1),
    "helmholtz_p1_513_x64": dict(N=513, omega=100.0, seed=1, nsrc=64,
                                 factor_dtype="c64"),
    # smaller parity cases (several tiles, ragged trees)
    "helmholtz_p1_17": dict(N=17, omega=4.0, seed=2, nsrc=2),
    "helmholtz_p1_33": dict(N=33, omega=8.0, seed=3, nsrc=3),
    "helmholtz_p1_129": dict(N=129, omega=32.0, seed=4, nsrc=4),
    "helmholtz_p1_257": dict(N=257, omega=50.0, seed=5, nsrc=8),
}


def make_problem(name, **overrides):
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    N = cfg.pop("N")
    omega = cfg.pop("omega")
    seed = cfg.pop("seed")
    nsrc = cfg.pop("nsrc")
    return _helmholtz(name, N, omega, seed, nsrc, **cfg)


@dataclass
class BatchProblem:
    """Uneven-sized independent problems solved together, each with its own
    seeded speed field, one Gaussian source, receivers and observed data."""
    name: str
    problems: list
    receivers: list               # per problem: int64 node ids
    data: list                    # per problem: complex128 (count, nrhs)


#: Batches of uneven problems.  The frequency of a grid of side N is
#: omega = kh (N - 1), so every problem resolves its shortest wavelength with
#: the same number of points (the speed is at least 1, so k h <= kh).
BATCHES = {
    "helmholtz_p1_batch256": dict(count=256, lo=65, hi=513, seed=0, kh=0.25, receivers=8),
    # reduced batches for parity tests
    "helmholtz_p1_batch8": dict(count=8, lo=9, hi=65, seed=8, kh=0.3, receivers=8),
    "helmholtz_p1_batch32": dict(count=32, lo=65, hi=129, seed=9, kh=0.2, receivers=8),
    # the 256-problem batch's size range and resolution on 16 problems
    "helmholtz_p1_batch16": dict(count=16, lo=65, hi=513, seed=0, kh=0.25, receivers=8),
}


def make_batch(name, device=None, **overrides):
    """The named batch; with a torch device the slowness fields are evaluated
    there and returned as tensors (the large batches would take minutes on
    the host)."""
    cfg = dict(BATCHES[name])
    cfg.update(overrides)
    count, seed = cfg["count"], cfg["seed"]
    Ns = batch_grid_sizes(seed, count, cfg["lo"], cfg["hi"])
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    problems, receivers, data = [], [], []
    for q, N in enumerate(int(v) for v in Ns):
        s = 1.0 / speed_field(N, seed * 100003 + q, device=device)
        f = gaussian_sources(N, source_centers(seed * 100003 + q, 1))
        problems.append(Problem(name=f"{name}[{q}]", N=N, omega=cfg["kh"] * (N - 1),
                                slowness=s, f=f, factor_dtype="c64"))
        receivers.append(receiver_nodes(N, seed * 100003 + q, cfg["receivers"]))
        d = rng.standard_normal((cfg["receivers"], 1)) + 1j * rng.standard_normal(
            (cfg["receivers"], 1))
        data.append(1e-4 * d)
    return BatchProblem(name=name, problems=problems, receivers=receivers, data=data)


def lame_fields(N, seed, ell=0.1, device=None):
    """Smooth Lame fields lam = 1 + 3*sigmoid(g1) in (1, 4) and
    mu = 0.5 + 1.5*sigmoid(g2) in (0.5, 2), g1, g2 the random fields of seeds
    seed and seed + 1; density rho = 1."""
    g1 = random_field(N, seed, ell, device=device)
    g2 = random_field(N, seed + 1, ell, device=device)
    if device is not None:
        import torch
        return (1.0 + 3.0 * torch.sigmoid(g1), 0.5 + 1.5 * torch.sigmoid(g2),
                torch.ones(N * N, dtype=torch.float64, device=device))
    sig = lambda g: 1.0 / (1.0 + np.exp(-g))  # noqa: E731
    return 1.0 + 3.0 * sig(g1), 0.5 + 1.5 * sig(g2), np.ones(N * N)


@dataclass
class ElasticProblem:
    """One seeded time-harmonic P1 elastic workload on [0,1]^2 with the
    first-order absorbing traction on all four sides.  Vectors hold
    2 * N * N entries, DOF id 2 * node + component (x, y)."""
    name: str
    N: int
    omega: float
    lam: np.ndarray               # (N*N,) nodal Lame lambda
    mu: np.ndarray                # (N*N,) nodal Lame mu
    rho: np.ndarray               # (N*N,) nodal density
    f: np.ndarray                 # (2*N*N, nrhs) nodal body-force samples
    leaf_dofs: int = 64
    beta: int = 32
    tol: float = 1e-6
    h_sw: int = 4
    gmres_m: int = 50
    gmres_tol: float = 1e-8
    factor_dtype: str = "c64"

    @property
    def n(self):
        return 2 * self.N * self.N

    @property
    def nrhs(self):
        return self.f.shape[1]


#: Elastic workloads: the 2.1M-DOF case at N = 1025 and small parity cases.
ELASTIC = {
    "elastic_p1_1025": dict(N=1025, omega=60.0, seed=0, nsrc=1),
    "elastic_p1_33": dict(N=33, omega=6.0, seed=2, nsrc=2),
    "elastic_p1_65": dict(N=65, omega=12.0, seed=4, nsrc=2),
    "elastic_p1_129": dict(N=129, omega=20.0, seed=6, nsrc=2),
    # coarser members of the 1025 family (omega scaled with N - 1)
    "elastic_p1_257": dict(N=257, omega=15.0, seed=0, nsrc=1),
    "elastic_p1_513": dict(N=513, omega=30.0, seed=0, nsrc=1),
}


def make_elastic(name, device=None, **overrides):
    """The named elastic workload: Lame fields from seeds (seed, seed + 1),
    vertical body forces (0, 1) times Gaussian bumps (width 0.02) at nsrc
    centres drawn with seed + 2.  With a torch device the Lame fields are
    evaluated there and returned as tensors."""
    cfg = dict(ELASTIC[name])
    cfg.update(overrides)
    N, seed, nsrc = cfg.pop("N"), cfg.pop("seed"), cfg.pop("nsrc")
    omega = float(cfg.pop("omega"))
    lam, mu, rho = lame_fields(N, seed, device=device)
    g = gaussian_sources(N, source_centers(seed + 2, nsrc))
    f = np.zeros((2 * N * N, nsrc))
    f[1::2] = g
    return ElasticProblem(name=name, N=N, omega=omega, lam=lam, mu=mu, rho=rho, f=f, **cfg)


def dg_node_coords(Nc):
    """(x, y) of the DOF nodes of the P2 discontinuous mesh: Nc x Nc cells of
    side 1/Nc, cell (i, j) split into the lower triangle (i,j), (i+1,j),
    (i+1,j+1) and the upper triangle (i,j), (i+1,j+1), (i,j+1); element
    2 (j Nc + i) + t holds its three vertices, then the midpoints of its
    edges (v0,v1), (v1,v2), (v2,v0).  Arrays of length 12 Nc^2."""
    h = 1.0 / Nc
    j, i = np.meshgrid(np.arange(Nc, dtype=np.float64), np.arange(Nc, dtype=np.float64),
                       indexing="ij")
    i, j = i.ravel(), j.ravel()
    lower = [(i, j), (i + 1, j), (i + 1, j + 1)]
    upper = [(i, j), (i + 1, j + 1), (i, j + 1)]
    out = np.empty((Nc * Nc, 2, 6, 2))
    for t, V in enumerate((lower, upper)):
        pts = V + [((V[0][0] + V[1][0]) / 2, (V[0][1] + V[1][1]) / 2),
                   ((V[1][0] + V[2][0]) / 2, (V[1][1] + V[2][1]) / 2),
                   ((V[2][0] + V[0][0]) / 2, (V[2][1] + V[0][1]) / 2)]
        for a, (px, py) in enumerate(pts):
            out[:, t, a, 0] = px * h
            out[:, t, a, 1] = py * h
    out = out.reshape(-1, 2)
    return out[:, 0], out[:, 1]


@dataclass
class DGProblem:
    """One seeded SIPG-P2 Helmholtz workload on [0,1]^2 with the absorbing
    condition on all four sides: slowness at the (Nc+1)^2 mesh vertices,
    sources sampled at the 12 Nc^2 DOF nodes."""
    name: str
    Nc: int
    omega: float
    slowness: np.ndarray          # ((Nc+1)^2,) vertex slowness s = 1/c
    f: np.ndarray                 # (12 Nc^2, nrhs) nodal source samples
    leaf_dofs: int = 60           # ND leaves of at most 10 triangles
    beta: int = 60                # HSS leaves of 10 triangles
    tol: float = 1e-4
    h_sw: int = 4
    gmres_m: int = 50
    gmres_tol: float = 1e-8
    factor_dtype: str = "c64"

    @property
    def n(self):
        return 12 * self.Nc * self.Nc

    @property
    def nrhs(self):
        return self.f.shape[1]


#: SIPG-P2 workloads: 256 x 256 x 2 triangles (786,432 DOFs) and parity cases
#: at the same resolution per cell (omega = 80 Nc / 256).
DG = {
    "sipg_p2_256": dict(Nc=256, omega=80.0, seed=0, nsrc=1),
    "sipg_p2_8": dict(Nc=8, omega=2.5, seed=3, nsrc=2),
    "sipg_p2_16": dict(Nc=16, omega=5.0, seed=4, nsrc=2),
    "sipg_p2_32": dict(Nc=32, omega=10.0, seed=5, nsrc=2),
    "sipg_p2_64": dict(Nc=64, omega=20.0, seed=6, nsrc=2),
    "sipg_p2_128": dict(Nc=128, omega=40.0, seed=0, nsrc=1),
}


def make_dg(name, device=None, **overrides):
    """The named SIPG-P2 workload: speed c = 1 + 2 sigmoid(g) (seed) at the
    mesh vertices, Gaussian sources (width 0.02) at centres drawn with the
    same seed, sampled at the DOF nodes.  With a torch device the speed
    field is evaluated there (returned as a tensor)."""
    cfg = dict(DG[name])
    cfg.update(overrides)
    Nc, seed, nsrc = cfg.pop("Nc"), cfg.pop("seed"), cfg.pop("nsrc")
    omega = float(cfg.pop("omega"))
    s = 1.0 / speed_field(Nc + 1, seed, device=device)
    x, y = dg_node_coords(Nc)
    centers = source_centers(seed, nsrc)
    f = np.empty((x.size, nsrc))
    for q, (cx, cy) in enumerate(centers):
        f[:, q] = np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * 0.02 * 0.02))
    return DGProblem(name=name, Nc=Nc, omega=omega, slowness=s, f=f, **cfg)


# ---------------------------------------------------------------- IPDG-P1
@dataclass
class IpdgProblem:
    """The scaling workload of Sec. 4.6: IPDG with P1 elements on Nc x Nc x 2
    triangles of the unit square (n = 6 Nc^2 = 6 / h^2 DOFs), u = 0 on the
    whole boundary, constant source f = 1, constant wavenumber kappa = omega
    (s = 1); omega = 0 is the Poisson problem.  Solver settings of Sec. 4:
    HSS tolerance 1e-6, block size beta = 10 (p+1)(p+2)/2 = 30 DOFs, ND
    leaves of fewer than 10 elements, HSS arithmetic from 4 levels above the
    leaves, GMRES restarted every 10 iterations, tolerance 1e-9, at most 30
    iterations."""
    name: str
    Nc: int
    omega: float
    slowness: np.ndarray          # ((Nc+1)^2,) ones
    f: np.ndarray                 # (6 Nc^2, 1) ones: the source f = 1 at the DOF nodes
    p: int = 1
    bc: str = "dirichlet"
    leaf_dofs: int = 30
    beta: int = 30
    tol: float = 1e-6
    h_sw: int = 4
    gmres_m: int = 10
    gmres_tol: float = 1e-9
    gmres_maxit: int = 30
    factor_dtype: str = "c128"

    @property
    def n(self):
        return 6 * self.Nc * self.Nc

    @property
    def nrhs(self):
        return self.f.shape[1]


#: wavenumber of each family as a function of the cells per side Nc = 1/h:
#: Poisson, Helmholtz kappa = 10 (Table 2), and kappa h = 1/4, 1/2 (Table 3)
IPDG_FAMILIES = {
    "poisson": lambda Nc: 0.0,
    "helmholtz_k10": lambda Nc: 10.0,
    "helmholtz_kh025": lambda Nc: Nc / 4.0,
    "helmholtz_kh05": lambda Nc: Nc / 2.0,
}
#: the mesh widths 1/h of Tables 2-3
IPDG_INV_H = (22, 32, 45, 64, 90, 128, 181, 256, 362, 512)


def make_ipdg(family, Nc, **overrides):
    """The IPDG-P1 Dirichlet workload of `family` on Nc = 1/h cells per side."""
    omega = float(IPDG_FAMILIES[family](Nc))
    cfg = dict(name=f"ipdg_p1_{family}_{Nc}", Nc=Nc, omega=omega,
               slowness=np.ones((Nc + 1) ** 2), f=np.ones((6 * Nc * Nc, 1)))
    cfg.update(overrides)
    return IpdgProblem(**cfg)
