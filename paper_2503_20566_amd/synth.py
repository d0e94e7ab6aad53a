"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmark.

Draws random numbers only; it holds none of the method's arithmetic.  Both sides receive the
same draws:
  * tensor entries: i.i.d. standard normals scaled by 1/D (D = total bond dimension), one per
    parameter, for a parameter count each side computes from its own layout code;
  * configurations: i.i.d. uniform plaquette powers k_p in {0, .., N-1}, one (L-1) x (L-1) grid
    per sample; each side turns powers into link labels with its own code;
  * flip masks for Z2 are the same draw with N = 2;
  * matter occupations (hard-core bosons): a uniformly random set of n_bosons occupied vertices
    per sample; each side builds a Gauss-law configuration around them with its own code.

The workload table lists the lattices the tests and the benchmark run (shapes from the paper's
Z2 / Z3 / Z4 studies: bond dimension D = N * D_k with D_k = 2 on 16 x 16, chi = 3 D_k when the
paper's rule is used).
"""
import numpy as np

THETA_SEED = 1234
SAMPLE_SEED = 5678

WORKLOADS = {
    # name: (L, N, D_k, chi, J, h, batch[, sweeps: the batch is that many Metropolis sweeps of chains
    # started from Philox-drawn plaquette powers, else uniform plaquette powers])
    "z2_4x4_d2": dict(L=4, N=2, Dk=1, chi=16, J=1.0, h=0.5, batch=256),
    "z2_16x16_d4": dict(L=16, N=2, Dk=2, chi=16, J=1.0, h=0.3, batch=4096, sweeps=10),
    "z3_16x16_d6": dict(L=16, N=3, Dk=2, chi=36, J=1.0, h=0.4, batch=2048),
    "z4_32x32_d8": dict(L=32, N=4, Dk=2, chi=64, J=1.0, h=0.5, batch=1024),
    # the same lattice at the largest cutoff the kernels hold with D_k = 2 (chi * D_k = 72)
    "z4_32x32_d8_chi36": dict(L=32, N=4, Dk=2, chi=36, J=1.0, h=0.5, batch=1024),
}


def theta_normals(n_params, D, seed=THETA_SEED):
    """i.i.d. N(0, 1) / D entries, float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(n_params) / float(D)


def plaquette_powers(batch, L, N, seed=SAMPLE_SEED):
    """Uniform plaquette powers, uint8 [batch, L-1, L-1] indexed [b, py, px]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, N, size=(batch, L - 1, L - 1), dtype=np.uint8)


def gauge_matrices(count, Dk, orthogonal, seed):
    """Random well-conditioned Dk x Dk matrices (orthogonal, or identity plus a small random
    part) for gauge-transformation tests; float64 [count, Dk, Dk]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.standard_normal((count, Dk, Dk))
    if orthogonal:
        q, r = np.linalg.qr(A)
        return q * np.sign(np.diagonal(r, axis1=1, axis2=2))[:, None, :]
    return np.eye(Dk)[None] + 0.3 * A


def link_labels(L, N, seed):
    """Uniform link labels in {0, .., N-1}, uint8 [2, L, L] indexed [direction, y, x]; every slot
    is drawn, also the ones with no link at the lattice edge (callers zero those)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, N, size=(2, L, L), dtype=np.uint8)


def normals(shape, seed):
    """i.i.d. N(0, 1) float64 array of the given shape: synthetic per-sample data (log-derivative
    values, local energies, test vectors) for parity tests of the SR build and solve, so that both
    sides receive the same inputs without either computing them."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape)


def occupations(batch, L, n_bosons, seed=SAMPLE_SEED + 1):
    """Hard-core boson occupations, uint8 [batch, L, L] indexed [b, y, x]: n_bosons vertices per
    sample, a uniformly random subset (the first n_bosons of a random permutation)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros((batch, L * L), dtype=np.uint8)
    for b in range(batch):
        out[b, rng.permutation(L * L)[:n_bosons]] = 1
    return out.reshape(batch, L, L)
