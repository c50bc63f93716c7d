"""Seeded synthetic inputs for the Jacobi workloads.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no sweep, no residual, no source scaling).  Both the
device path's tests/benchmark and the CPU oracle receive the arrays it makes.

Every generator draws in FP64 from numpy's PCG64 (``numpy.random.default_rng``)
with the seed given; an FP32 run rounds the same values to FP32 once (the FP64
oracle then sees those rounded values widened back to FP64).

Workload recipes (the paper measures on no public data set; all inputs are
synthetic, shaped like the Jacobi3D proxy's domain of Section 4.3):
  laplace2d_top_edge   256^2 interior, ring: top edge (y = 1) = 1.0, other
                       edges and the corners 0.0; interior u_0 ~ U[0,1) from
                       default_rng(1).
  poisson2d_gaussians  8192^2 interior, f = sum of 16 Gaussians
                       (default_rng(2)), zero ring, u_0 = 0.
  poisson3d_uniform    512^3 interior, f ~ U[-1,1) (default_rng(3)), zero
                       ring, u_0 = 0.
  batched_sizes / batched_source
                       64 grids, sides n_g ~ integers in [257, 4097] from
                       default_rng(4); f_g Gaussian sums from
                       default_rng(4000+g); zero ring, u_0 = 0.
  adjoint_gaussians    4096^2, f and target Gaussian sums (default_rng(5),
                       (6)); ring values ~ U[0,1) on non-corner ring nodes
                       (default_rng(7)), corners 0; u_0 = 0;
                       finite-difference picks from default_rng(8).
"""
import numpy as np


def spacing2(n):
    """Squared mesh spacing h^2 of the unit interval cut by n interior nodes,
    h = 1/(n+1): one FP64 rounding of 1/(n+1)^2."""
    return 1.0 / float((n + 1) * (n + 1))


def node_coords(n):
    """Coordinates x_i = i*h of interior nodes i = 1..n (FP64)."""
    return np.arange(1, n + 1, dtype=np.float64) / float(n + 1)


def gaussian_sum(n, ndim, seed, count=16):
    """f(x) = sum_m A_m exp(-|x - c_m|^2 / (2 sigma_m^2)) at interior nodes.

    Per Gaussian, drawn in this order from default_rng(seed): the centre
    coordinates (x, y[, z]) ~ U[0,1), sigma ~ U[0.01, 0.05], A ~ N(0,1).
    Returns an FP64 array of shape (n,)*ndim, x fastest (last axis)."""
    rng = np.random.default_rng(seed)
    params = []
    for _ in range(count):
        c = rng.random(ndim)
        sigma = rng.uniform(0.01, 0.05)
        amp = rng.standard_normal()
        params.append((c, sigma, amp))
    x = node_coords(n)
    f = np.zeros((n,) * ndim, dtype=np.float64)
    for c, sigma, amp in params:
        inv = 1.0 / (2.0 * sigma * sigma)
        # separable factors exp(-(x-cx)^2 inv) per axis; x is the last axis
        factors = [np.exp(-((x - c[a]) ** 2) * inv) for a in range(ndim)]
        if ndim == 2:
            f += amp * np.outer(factors[1], factors[0])
        else:
            f += amp * (factors[2][:, None, None] * factors[1][None, :, None]
                        * factors[0][None, None, :])
    return f


def uniform(shape, seed, lo=0.0, hi=1.0):
    """U[lo, hi) in FP64 from default_rng(seed), C order."""
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def state_with_ring(interior, ring=None):
    """Full node array: interior values inside, ring values (same-shaped full
    array whose interior is ignored) or zero outside."""
    interior = np.asarray(interior, dtype=np.float64)
    shape = tuple(s + 2 for s in interior.shape)
    U = np.zeros(shape, dtype=np.float64) if ring is None else np.array(ring, dtype=np.float64)
    U[(slice(1, -1),) * interior.ndim] = interior
    return U


def laplace2d_top_edge(n=256, seed=1):
    """256^2 Laplace case: ring top edge (row y index n+1) = 1.0, else 0; u_0 ~ U[0,1)."""
    U = np.zeros((n + 2, n + 2), dtype=np.float64)
    U[n + 1, 1:n + 1] = 1.0
    U[1:n + 1, 1:n + 1] = uniform((n, n), seed)
    return U


def poisson2d_gaussians(n=8192, seed=2):
    """Config 2: returns (U0 zero everywhere, f Gaussian sum)."""
    return np.zeros((n + 2, n + 2), dtype=np.float64), gaussian_sum(n, 2, seed)


def poisson3d_uniform(n=512, seed=3):
    """Config 3: returns (U0 zero, f ~ U[-1,1))."""
    return (np.zeros((n + 2,) * 3, dtype=np.float64), uniform((n, n, n), seed, -1.0, 1.0))


def batched_sizes(count=64, seed=4, lo=257, hi=4097):
    """Config 4 side lengths: integers uniform on [lo, hi] inclusive."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=count).astype(np.int64)


def batched_source(n, g, base_seed=4000):
    """Config 4 source of grid g: 16-Gaussian sum from default_rng(base + g)."""
    return gaussian_sum(n, 2, base_seed + g)


def ring_values(n, ndim, seed):
    """Full zero array whose non-corner ring nodes are U[0,1) from default_rng(seed).

    Draw order: the ring nodes of the full array in C order."""
    shape = (n + 2,) * ndim
    U = np.zeros(shape, dtype=np.float64)
    mask = ring_mask(n, ndim)
    vals = np.random.default_rng(seed).random(int(mask.sum()))
    U[mask] = vals
    return U


def ring_mask(n, ndim):
    """Boolean mask of non-corner ring nodes (nodes with exactly one coordinate
    on the boundary in 2D; with exactly one in 3D as well, i.e. face nodes)."""
    idx = np.indices((n + 2,) * ndim)
    on = sum(((a == 0) | (a == n + 1)).astype(np.int64) for a in idx)
    return on == 1


def adjoint_gaussians(n=4096):
    """Config 5: returns (U0 with ring ~ U[0,1) and zero interior, f, target)."""
    U0 = ring_values(n, 2, 7)
    f = gaussian_sum(n, 2, 5)
    t = gaussian_sum(n, 2, 6)
    return U0, f, t


def fd_picks(n, count=32, seed=8, ndim=2):
    """Finite-difference entry picks: `count` interior cells of f and `count`
    non-corner ring nodes, without replacement, from default_rng(seed).
    Returns (list of interior index tuples, list of full-array ring index tuples)."""
    rng = np.random.default_rng(seed)
    cells = rng.choice(n ** ndim, size=count, replace=False)
    f_idx = [tuple(int(v) for v in np.unravel_index(c, (n,) * ndim)) for c in cells]
    ring_nodes = np.argwhere(ring_mask(n, ndim))
    picks = rng.choice(len(ring_nodes), size=count, replace=False)
    g_idx = [tuple(int(v) for v in ring_nodes[p]) for p in picks]
    return f_idx, g_idx
