"""Real-time evolution by time-dependent VMC with complex tensors (oracle; test infrastructure only).

Paper passages followed:
  * SM S-3 eq. tVMC: i S_mn alphadot_n = g_m with S_mn = <O*_m O_n> - <O*_m><O_n> (SM S-3, S_mn),
    solved for alphadot (the paper iterates CG; here a dense library solve of the same system, with
    an optional diagonal shift, or the minimum-norm least-squares solution);
  * SM S-1 eq. gradient, read as the covariance g_m = <O*_m E_loc> - <O*_m><E_loc>;
  * SM S-3 eq. secondorder: two updates per time step, with c_{1,2} = (1 +- i)/2;
  * SM S-1 eq. Es: E_loc(s) = sum_{s'} <s|H|s'> Psi(s') / Psi(s), here with complex ratios.

Readings (the paper leaves these open):
  * O_m = d ln Psi / d alpha_m, the holomorphic derivative of the amplitude of complex tensors.  A
    truncated SVD is not holomorphic, so this oracle contracts the network exactly (bond dimension
    not truncated: small lattices); Psi is then multilinear in the site tensors and d Psi / dT_x is
    the network with site x's legs left open.
  * Expectations are exact sums over the physical configurations with weights |Psi|^2 / sum |Psi|^2
    (no sampling).
  * Direction of time: with O, S and g as above, the solution of i S alphadot = g is d alpha / dt
    of the time-dependent variational principle for i d|psi>/dt = H|psi>.  The printed update
    subtracts Delta t * alphadot, which under these conventions steps backwards; each stage here
    adds c Delta t alphadot (alpha <- alpha + c_1 dt alphadot(alpha), then with c_2), and the pins
    against exact evolution fix the direction.  With c_1 + c_2 = 1 and c_1 c_2 = 1/2 the two stages
    reproduce exp(A dt) of linear dynamics to second order.
"""
import numpy as np

from .energy import electric_energy
from .lattice import apply_plaquette
from .layout import project


def _network(tensors, open_site=None):
    """einsum operands of the whole network (tensors[y][x] with legs (l, r, d, u), absent legs of
    dimension 1); with open_site = (x, y) that tensor is left out and its present legs are the
    output indices, in (l, r, d, u) order."""
    L = len(tensors)
    lab = {}

    def label(key):
        if key not in lab:
            lab[key] = len(lab)
        return lab[key]

    operands, out = [], []
    for y in range(L):
        for x in range(L):
            T = tensors[y][x]
            subs = []
            keep = []
            for leg, key in enumerate((("h", x - 1, y), ("h", x, y), ("v", x, y - 1), ("v", x, y))):
                if (x > 0, x < L - 1, y > 0, y < L - 1)[leg]:
                    keep.append(leg)
                    subs.append(label(key))
            if open_site == (x, y):
                out = subs
                continue
            idx = tuple(slice(None) if leg in keep else 0 for leg in range(4))
            operands.append(T[idx])
            operands.append(subs)
    return operands, out


def exact_amplitude(tensors):
    """Psi of the projected network of complex tensors, contracted exactly (numpy.einsum)."""
    operands, _ = _network(tensors)
    return complex(np.einsum(*operands, [], optimize="greedy"))


def log_derivatives(layout, theta, links):
    """Dense O[n_params] = d ln Psi / d theta (complex): nonzero on each site's selected block,
    where it is (network with that site's legs open) / Psi."""
    ok, T, bid = project(layout, theta, links)
    assert ok
    psi = exact_amplitude(T)
    L = layout.L
    O = np.zeros(layout.n_params, dtype=complex)
    for y in range(L):
        for x in range(L):
            operands, out = _network(T, open_site=(x, y))
            env = np.einsum(*operands, out, optimize="greedy") if operands else np.ones(())
            _, shape, off = layout.blocks[layout.site(x, y)][bid[y, x]]
            O[off: off + int(np.prod(shape))] = np.asarray(env).reshape(-1) / psi
    return O


def amplitude_of(layout, theta):
    def f(links):
        ok, T, _ = project(layout, theta, links)
        return exact_amplitude(T) if ok else 0.0
    return f


def local_energy(layout, theta, links, c_tab, e_tab, amp=None):
    """E_loc(s) with complex amplitude ratios of the exact contraction (eq. Es)."""
    L, N = layout.L, layout.N
    amp = amp or amplitude_of(layout, theta)
    psi = amp(links)
    tot = complex(electric_energy(links, e_tab))
    for py in range(L - 1):
        for px in range(L - 1):
            for t in range(1, N):
                if c_tab[t] != 0.0:
                    tot += c_tab[t] * amp(apply_plaquette(links, px, py, (N - t) % N, N)) / psi
    return tot


def state_vector(layout, theta, configs):
    """Psi(s) over a list of configurations (the basis of an exact-evolution comparison)."""
    f = amplitude_of(layout, theta)
    return np.array([f(s) for s in configs], dtype=complex)


def tdvp_rhs(layout, theta, configs, c_tab, e_tab, shift=0.0, rcond=None, weights="psi2"):
    """alphadot solving i S alphadot = g over the configurations.

    weights "psi2": exact weights |Psi|^2 / sum |Psi|^2 (the configurations enumerate the space);
    "uniform": plain means over the configurations, the Monte Carlo average of SM S-1 / S-3 when
    they are samples drawn from |Psi|^2.
    shift > 0: dense solve of i (S + shift I) alphadot = g; else the minimum-norm least-squares
    solution (numpy.linalg.lstsq with rcond).  Returns (alphadot, <H>, S, g)."""
    amp = amplitude_of(layout, theta)
    psi = np.array([amp(s) for s in configs], dtype=complex)
    if weights == "uniform":
        p = np.full(len(configs), 1.0 / len(configs))
    else:
        w = np.abs(psi) ** 2
        p = w / w.sum()
    O = np.array([log_derivatives(layout, theta, s) for s in configs])
    E = np.array([local_energy(layout, theta, s, c_tab, e_tab, amp) for s in configs])
    Om = p @ O
    Em = complex(p @ E)
    S = (O.conj().T * p) @ O - np.outer(Om.conj(), Om)
    g = (O.conj().T * p) @ E - Om.conj() * Em
    if shift > 0.0:
        x = np.linalg.solve(1j * (S + shift * np.eye(S.shape[0])), g)
    else:
        x = np.linalg.lstsq(1j * S, g, rcond=rcond)[0]
    return x, Em.real, S, g


def step(layout, theta, configs, c_tab, e_tab, dt, order=2, **solve):
    """One time step: eq. secondorder (two stages, c_{1,2} = (1 +- i)/2) or, for order=1, the
    single Euler stage alpha + dt alphadot.  Returns (theta(t + dt), <H>(t))."""
    x, eh, _, _ = tdvp_rhs(layout, theta, configs, c_tab, e_tab, **solve)
    if order == 1:
        return theta + dt * x, eh
    c1, c2 = (1 + 1j) / 2, (1 - 1j) / 2
    t1 = theta + c1 * dt * x
    x1, _, _, _ = tdvp_rhs(layout, t1, configs, c_tab, e_tab, **solve)
    return t1 + c2 * dt * x1, eh


def evolve(layout, theta0, configs, c_tab, e_tab, dt, n_steps, order=2, **solve):
    """theta(t) and <H>(t) for t = 0, dt, ..., n_steps dt."""
    thetas = [np.asarray(theta0, dtype=complex)]
    energies = []
    for _ in range(n_steps):
        th, eh = step(layout, thetas[-1], configs, c_tab, e_tab, dt, order=order, **solve)
        thetas.append(th)
        energies.append(eh)
    energies.append(tdvp_rhs(layout, thetas[-1], configs, c_tab, e_tab, **solve)[1])
    return thetas, np.array(energies)
