"""Seeded synthetic inputs for the NFFT workloads.

This module only draws random numbers and lays them out; it holds none of the
transform's arithmetic, so the oracle and the HIP path can both take their
inputs from here.

Workloads (sizes from the evaluation plan; node layouts as stated):

* ``"paper"``: the test polynomials of Sec. 4 eq. (4.1): coefficients
  1 / (1 + ||k||_2) on I_N and nodes uniform on [-1/2, 1/2)^d.
* ``"d1"``:   d=1, N=256, M=1024, uniform nodes, complex Gaussian data.
* ``"d2"``:   d=2, N=(512,512), M=262144, uniform nodes, complex Gaussian data.
* ``"d3r"``:  d=3, N=(128,128,128), M=4096*512 nodes on full-diameter radial spokes
  (directions uniform on the sphere), complex Gaussian data.
* ``"batch"``: 64 independent d=2 plans, N_t drawn from {64,128,256,512} per
  dimension, M log-uniform in [1e3, 2e5], uniform nodes.
* ``"grad"``: d=2, N=(256,256), M=256 spokes * 256 points with N(0, 1e-3^2) jitter.
* ``"fastsum"``: d=2, N=(128,128), 32768 source and 32768 target nodes, uniform.
* ``"nnfft_d2"``: NNFFT, d=2, N=(256,256): K=131072 frequencies uniform on
  [-128, 128)^2 and M=131072 nodes uniform on [-1/2, 1/2)^2, m=8, complex Gaussian data.

"Complex Gaussian" is CN(0,1): (a + i b)/sqrt(2) with a, b standard normal.
Seeds are 18100989100 + 10*workload_id + stream_id, PCG64.
"""
import numpy as np

SEED_BASE = 18100989100

WORKLOAD_ID = {"d1": 1, "d2": 2, "d3r": 3, "batch": 4, "grad": 5, "paper": 6, "small": 7, "fastsum": 8, "nnfft_d2": 9}


def rng(workload, stream=0):
    return np.random.default_rng(SEED_BASE + 10 * WORKLOAD_ID[workload] + stream)


def cgauss(r, shape):
    """CN(0,1) samples of the given shape (complex128)."""
    a = r.standard_normal(shape)
    b = r.standard_normal(shape)
    return (a + 1j * b) / np.sqrt(2.0)


def uniform_nodes(r, M, d):
    """M nodes uniform on [-1/2, 1/2)^d, float64, shape (M, d)."""
    return r.random((M, d)) - 0.5


def paper_coefficients(N):
    """1/(1 + ||k||_2) on the centred index set I_N (Sec. 4 eq. (4.1))."""
    grids = np.meshgrid(*[np.arange(-v // 2, v // 2) for v in N], indexing="ij")
    k2 = np.zeros(tuple(N))
    for g in grids:
        k2 = k2 + g.astype(np.float64) ** 2
    return (1.0 / (1.0 + np.sqrt(k2))).astype(np.complex128)


def radial_nodes_3d(r, spokes, points):
    """Full-diameter spokes through the origin: direction v_s uniform on the sphere,
    point i at ((i - points/2) / points) * v_s, i = 0..points-1, so every coordinate
    lies in [-1/2, 1/2).  Shape (spokes*points, 3)."""
    v = r.standard_normal((spokes, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    t = (np.arange(points) - points // 2) / float(points)
    x = t[None, :, None] * v[:, None, :]
    return np.ascontiguousarray(x.reshape(-1, 3))


def radial_nodes_2d(r, spokes, points, jitter):
    """Spoke s at angle pi*s/spokes, point i at t_i = (i - points/2)/points, plus
    N(0, jitter^2) noise per coordinate, wrapped into [-1/2, 1/2)."""
    th = np.pi * np.arange(spokes) / spokes
    t = (np.arange(points) - points // 2) / float(points)
    x = np.stack([t[None, :] * np.cos(th)[:, None], t[None, :] * np.sin(th)[:, None]], axis=-1)
    x = x.reshape(-1, 2) + jitter * r.standard_normal((spokes * points, 2))
    x = (x + 0.5) % 1.0 - 0.5
    return np.ascontiguousarray(x)


def workload(name, m=None, stream=0):
    """Inputs of one named workload: dict with N, M, n (None = default), m, x, fhat, f."""
    r = rng(name, stream)
    if name == "d1":
        N, M = (256,), 1024
        x = uniform_nodes(r, M, 1)
        m = 8 if m is None else m
    elif name == "d2":
        N, M = (512, 512), 262144
        x = uniform_nodes(r, M, 2)
        m = 8 if m is None else m
    elif name == "d3r":
        N = (128, 128, 128)
        x = radial_nodes_3d(r, 4096, 512)
        M = x.shape[0]
        m = 6 if m is None else m
    elif name == "grad":
        N = (256, 256)
        x = radial_nodes_2d(r, 256, 256, 1e-3)
        M = x.shape[0]
        m = 6 if m is None else m
    elif name == "nnfft_d2":
        N, K, M = (256, 256), 131072, 131072
        m = 8 if m is None else m
        x = uniform_nodes(r, M, 2)
        v = (r.random((K, 2)) - 0.5) * np.asarray(N, dtype=np.float64)
        return {"N": N, "K": K, "M": M, "m": m, "x": x, "v": v, "fhat": cgauss(r, (K,)), "f": cgauss(r, (M,))}
    else:
        raise ValueError(name)
    fhat = cgauss(r, N)
    f = cgauss(r, (M,))
    return {"N": N, "M": M, "n": tuple(2 * v for v in N), "m": m, "x": x, "fhat": fhat, "f": f}


def paper_workload(d, stream=0):
    """Sec. 4 test polynomial f_d: N = 512 / (128,128) / (32,32,32), M = 2*prod(N)."""
    N = {1: (512,), 2: (128, 128), 3: (32, 32, 32)}[d]
    M = 2 * int(np.prod(N))
    r = rng("paper", stream * 4 + d)
    return {"N": N, "M": M, "x": uniform_nodes(r, M, d), "fhat": paper_coefficients(N)}


def batch_plans(count=64, stream=0):
    """Plan list of the batched workload: list of dicts with N, M, x, fhat, f."""
    r = rng("batch", stream)
    sizes = np.array([64, 128, 256, 512])
    plans = []
    for _ in range(count):
        N = (int(r.choice(sizes)), int(r.choice(sizes)))
        M = int(round(float(np.exp(r.uniform(np.log(1e3), np.log(2e5))))))
        plans.append({"N": N, "M": M})
    for p in plans:
        p["x"] = uniform_nodes(r, p["M"], 2)
        p["fhat"] = cgauss(r, p["N"])
        p["f"] = cgauss(r, (p["M"],))
    return plans


def small_case(d, N, M, seed=0, kind="uniform"):
    """Small seeded case for parity tests: nodes of the given kind, CN(0,1) data."""
    r = np.random.default_rng(SEED_BASE + 10 * WORKLOAD_ID["small"] + seed)
    if kind == "uniform":
        x = uniform_nodes(r, M, d)
    elif kind == "clustered":
        x = 0.02 * r.standard_normal((M, d))
        x = (x + 0.5) % 1.0 - 0.5
    elif kind == "wide":
        x = 3.0 * (r.random((M, d)) - 0.5)  # nodes outside [-1/2,1/2), treated periodically
    else:
        raise ValueError(kind)
    return {"x": np.ascontiguousarray(x), "fhat": cgauss(r, tuple(N)), "f": cgauss(r, (M,))}
