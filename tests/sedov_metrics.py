"""Shape of a Sedov blast on a uniform grid against the self-similar
solution (sedov_similarity.py): the density-profile L1 error, the radius of
the shell-averaged density peak, the density peaks along a coordinate axis
and a body diagonal (a grid-aligned error shows there) and the angular
scatter of the density in the shells near the shock.  Test support only."""
import numpy as np

import sedov_similarity as ss


def exact_density(r, R, gamma):
    lam, (U, G, P) = ss.solve(gamma)
    order = np.argsort(lam)
    x = r / R
    inside = np.interp(x, lam[order], G[order])
    return np.where(x < 1.0, inside, 1.0)


def end_time(R, gamma):
    """Time at which the shock of a unit-energy blast in unit density reaches R."""
    return (R / ss.xi0(gamma)) ** 2.5


def metrics(tree, U, R, gamma):
    xc = tree.cell_centres()                                  # [n, 3, E, E, E]
    r = np.sqrt((xc ** 2).sum(axis=1)).ravel()
    rho = U[:, 0].ravel()
    ex = exact_density(r, R, gamma)
    l1 = np.abs(rho - ex).sum() / ex.sum()
    dx = tree.dx0
    edges = np.arange(0.0, 0.5, dx)
    idx = np.digitize(r, edges)
    prof = np.array([rho[idx == i].mean() for i in range(1, len(edges))])
    rc = 0.5 * (edges[1:] + edges[:-1])
    r_peak = rc[np.argmax(prof)]
    X = xc[:, 0].ravel()
    Y = xc[:, 1].ravel()
    Z = xc[:, 2].ravel()
    h = 0.5 * dx + 1e-12
    axis = (np.abs(Y) <= h) & (np.abs(Z) <= h) & (X > 0)
    diag = (np.abs(X - Y) <= 1e-12) & (np.abs(X - Z) <= 1e-12) & (X > 0)
    shells = [i for i in range(1, len(edges)) if abs(rc[i - 1] - R) <= 0.25 * R]
    scatter = float(np.mean([rho[idx == i].std() / rho[idx == i].mean() for i in shells]))
    return dict(l1=l1, r_peak=r_peak, r_axis=r[axis][np.argmax(rho[axis])],
                r_diag=r[diag][np.argmax(rho[diag])], rho_max=rho.max(), R=R,
                rho_axis=rho[axis].max(), rho_diag=rho[diag].max(), scatter=scatter)


def describe(name, d, steps):
    return (f"{name}: density L1 {d['l1']:.4f}; shock radius {d['r_peak']:.4f} (exact {d['R']}); "
            f"peak along axis {d['r_axis']:.4f} / diagonal {d['r_diag']:.4f}, peak density there "
            f"{d['rho_axis']:.3f} / {d['rho_diag']:.3f}; shell scatter {d['scatter']:.4f}; "
            f"peak density {d['rho_max']:.3f}; {steps} steps")
