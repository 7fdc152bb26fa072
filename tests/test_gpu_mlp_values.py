"""Element-wise parity of the learned reconstruction's inference pre-pass
(hydro_mlp_values) and of the learned stage, against the CPU oracle.

Two kinds of network:

* A network whose output layer has zero weights, so that its outputs are its
  output biases exactly on both sides (the bfloat16 MFMA products are zeros,
  the FP32 accumulator starts from the bias; the oracle's FP64 sum is zero
  plus the bias, rounded to binary32).  Everything after the network -- the
  FP64 de-normalisation q_c + sigma y, the plain limiter, the FP64 check, the
  per-cell fallback and the fluxes built from the values -- is then the same
  arithmetic on the same numbers, so point values and verdicts must agree
  bit for bit, and the learned stage within the FP64 parity bound.
* Networks with all weights non-zero (random, and trained on plain-PPM
  pairs).  The two sides accumulate the layers in different orders and
  precisions (FP32 MFMA against an FP64 sum rounded to binary32) and evaluate
  GELU differently (hardware exp2/rcp against FP64 tanh), so a bfloat16
  activation can round to a neighbouring value on one side: each such flip
  moves an output by about |W3| 2^-8 |a|.  Raw outputs are compared element by
  element against a bound derived from that; point values within
  2 sigma max|dy| of the row (the limiter's clamp is 1-Lipschitz, the
  constraint 3 q_c - 2 R at most 2-Lipschitz) plus the binary32 rounding
  of offsets from q_c of at most 2 sigma on each side, except lines that one side
  flattens at an extremum while the other has an end within that distance of
  q_c (the constraint's only discontinuity); cell verdicts may differ only on
  a small counted set of cells.

Grids: an 85-leaf periodic two-level mesh with a smooth random state (every row
non-flat; same-level, injected and 2^3-mean ghosts), the 4096-leaf rotating
polytrope (star edge: the density-contrast rule; 1e-10 atmosphere) on
sampled leaves, and 16^3 leaves (eight tiles each) on an AMR mesh."""
import concurrent.futures as cf

import numpy as np
import pytest

import parity
from paper_2107_10987_amd.workloads import (PERIODIC, LeafSet, conserved_from_primitive,
                                            rotating_polytrope, split_octets, to_tiles8)

pytestmark = pytest.mark.gpu
NS = 896


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


# -- workloads -----------------------------------------------------------------

def _smooth_state(tree, seed=5, gamma=5.0 / 3.0):
    rng = np.random.default_rng(seed)
    x = tree.cell_centres()
    ph = rng.uniform(0, 2 * np.pi, size=6)
    r2 = ((x[:, 0] - 0.45) ** 2 + (x[:, 1] - 0.5) ** 2 + (x[:, 2] - 0.55) ** 2)
    rho = 1.0 + 2.0 * np.exp(-r2 / 0.02) + 0.2 * np.sin(2 * np.pi * x[:, 1] + ph[0])
    vx = 0.5 + 0.3 * np.sin(2 * np.pi * (x[:, 1] + x[:, 2]) + ph[1])
    vy = -0.4 + 0.2 * np.sin(2 * np.pi * (x[:, 0] + x[:, 2]) + ph[2])
    vz = 0.3 * np.sin(2 * np.pi * (x[:, 0] + x[:, 1]) + ph[3])
    p = 1.0 + 0.5 * np.exp(-r2 / 0.03) + 0.1 * np.sin(2 * np.pi * x[:, 0] + ph[4])
    spc = rho * (0.5 + 0.4 * np.sin(2 * np.pi * x[:, 2] + ph[5]))
    E = tree.leaf_edge
    U = conserved_from_primitive(rho, vx, vy, vz, p, spc, gamma)
    return np.ascontiguousarray(U.reshape(tree.n, 7, E, E, E))


def _amr32():
    ls = LeafSet((4, 4, 4), (PERIODIC,) * 3, (0.0, 0.0, 0.0), 1.0 / 32,
                 [(0, i, j, k) for i in range(4) for j in range(4) for k in range(4)])
    ls.refine(0, (1, 1, 1))
    ls.refine(0, (2, 1, 1))
    ls.refine(0, (3, 3, 2))
    return ls.tree()


def _amr16():
    ls = LeafSet((2, 2, 2), (PERIODIC,) * 3, (0.0, 0.0, 0.0), 1.0 / 32,
                 [(0, i, j, k) for i in range(2) for j in range(2) for k in range(2)], leaf_edge=16)
    ls.refine(0, (0, 0, 0))
    ls.refine(0, (1, 1, 1))
    return ls.tree()


class Case:
    """tree (as the library sees it), state, the oracle's 8^3-leaf tree and
    state, leaf edge, and the 8^3 blocks to check."""

    def __init__(self, name):
        import oracle
        self.name = name
        if name == "amr32":
            self.tree = _amr32()
            self.U = _smooth_state(self.tree)
            self.t8, self.U8 = self.tree, self.U
            self.edge, self.omega = 8, 0.0
            self.blocks = np.arange(self.tree.n)
        elif name == "polytrope":
            w = rotating_polytrope()
            self.tree, self.U, self.omega = w.tree, w.U, w.omega
            self.t8, self.U8, self.edge = w.tree, w.U, 8
            self.blocks, self.edge_leaves = _polytrope_sample(w)
        elif name == "leaf16":
            self.tree = _amr16()
            self.U = _smooth_state(self.tree, seed=7)
            self.t8, self.U8 = split_octets(self.tree), to_tiles8(self.U)
            self.edge, self.omega = 16, 0.0
            self.blocks = np.sort(np.random.default_rng(3).choice(self.t8.n, 48, replace=False))
        else:
            raise ValueError(name)
        self.ora = oracle.Oracle(self.t8, 5.0 / 3.0, self.omega)


def _polytrope_sample(w):
    """48 leaves: 16 with 2^3-mean ghosts (a finer neighbour), 16 with
    injected ghosts (a coarser neighbour), 16 straddling the star's edge."""
    from paper_2107_10987_amd.hydro import ghost_map
    gm = ghost_map(w.tree)
    lev = w.tree.level
    has_mean = (gm < 0).any(axis=1)
    src = np.where(gm >= 0, gm // 512, np.arange(w.n)[:, None])
    has_inj = (lev[src] < lev[:, None]).any(axis=1)
    rho = w.U[:, 0].reshape(w.n, -1)
    edge = (rho.max(axis=1) > 1e-6) & (rho.min(axis=1) < 1e-8)
    rng = np.random.default_rng(4)
    pick = []
    for sel in (has_mean & ~has_inj, has_inj, edge):
        cand = np.setdiff1d(np.flatnonzero(sel), pick)
        pick += list(rng.choice(cand, 16, replace=False))
    return np.sort(np.array(pick)), np.flatnonzero(edge)


# -- slot <-> oracle cell ------------------------------------------------------

def _slot_cells():
    """Oracle cell index ((k+1)*100 + (j+1)*10 + (i+1)) of each of the 896 slots."""
    out = np.empty(NS, np.int64)
    for s in range(NS):
        if s < 512:
            i, j, k = s & 7, (s >> 3) & 7, s >> 6
        else:
            slab, r = divmod(s - 512, 64)
            u, v = r & 7, r >> 3
            side = -1 if slab % 2 == 0 else 8
            if slab < 2:
                i, j, k = side, u, v
            elif slab < 4:
                i, j, k = u, side, v
            else:
                i, j, k = u, v, side
        out[s] = (k + 1) * 100 + (j + 1) * 10 + (i + 1)
    return out


SLOT_CELL = _slot_cells()
# the 13 lines as (index of +d, index of -d) in the 26-point numbering
LINES = []
for _d in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1),
           (0, 1, -1), (1, 1, 1), (1, 1, -1), (1, -1, 1), (1, -1, -1)]:
    _p = 9 * (_d[2] + 1) + 3 * (_d[1] + 1) + (_d[0] + 1)
    _m = 26 - _p
    LINES.append((_p if _p < 13 else _p - 1, _m if _m < 13 else _m - 1))
LINES = np.array(LINES)


def _sigma_qc(P):
    """sigma and q_c of every row [1000][7] of one padded block [7][14][14][14]."""
    c = P[:, 2:12, 2:12, 2:12]
    sig = np.zeros_like(c)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                nb = P[:, 2 + dz:12 + dz, 2 + dy:12 + dy, 2 + dx:12 + dx]
                sig = np.maximum(sig, np.abs(nb - c))
    return sig.reshape(7, 1000).T, c.reshape(7, 1000).T


def _oracle_rows(case, params):
    """Oracle rows of the checked blocks: dict block -> (y, val, ok, flat, sigma, qc)."""
    import oracle
    P = case.ora.padded(case.U8)

    def one(b):
        y, val, ok, flat = oracle.learned_rows(P[b], params)
        sig, qc = _sigma_qc(P[b])
        return int(b), (y, val, ok, flat, sig, qc)

    with cf.ThreadPoolExecutor(8) as ex:
        return dict(ex.map(one, case.blocks))


def _gpu_values(torch, case, params, want_y):
    """The pre-pass over the whole mesh; values, verdicts and raw outputs of
    the checked blocks, keyed by block."""
    from paper_2107_10987_amd.hydro import Hydro
    hy = Hydro(max_leaves=case.tree.n, learned=True, leaf_edge=case.edge)
    try:
        hy.mlp_load(params)
        g = hy.grid(case.tree, torch.tensor(case.U, device="cuda"), case.omega, 5.0 / 3.0)
        val, ok, y = hy.mlp_values(g, want_y=want_y)
        idx = torch.tensor(case.blocks, device="cuda")
        val, ok = val.index_select(0, idx).cpu().numpy(), ok.index_select(0, idx).cpu().numpy()
        y = None if y is None else y.index_select(0, idx).cpu().numpy()
        del g
    finally:
        hy.close()
    keys = [int(b) for b in case.blocks]
    return (dict(zip(keys, val)), dict(zip(keys, ok.astype(bool))),
            None if y is None else dict(zip(keys, y)))


def _constant_network(seed=11, scale=0.6):
    rng = np.random.default_rng(seed)
    p = (rng.normal(size=8090) * 0.3).astype(np.float32)
    p[6400:8064] = 0.0                                  # W3: outputs = b3 exactly
    p[8064:] = rng.uniform(-scale, scale, 26).astype(np.float32)
    return p


CASES = {}


def _case(name):
    if name not in CASES:
        CASES[name] = Case(name)
    return CASES[name]


# -- bitwise: constant-output network ------------------------------------------

@pytest.mark.parametrize("name", ["amr32", "polytrope", "leaf16"])
def test_constant_network_values_and_verdicts_bitwise(torch, name):
    case = _case(name)
    p = _constant_network()
    print(f"case: pre-pass values, constant-output network, {name}, {len(case.blocks)} blocks", flush=True)
    val, ok, _ = _gpu_values(torch, case, p, want_y=False)
    rows = _oracle_rows(case, p)
    nfail = nflat_cell = 0
    for b, (_, oval, rok, flat, sig, qc) in rows.items():
        ovals = oval[SLOT_CELL]                            # [896][7][26]
        cell_ok = rok[SLOT_CELL].all(axis=1)               # [896]
        assert np.array_equal(ok[b].astype(bool), cell_ok), (name, b)
        g = val[b].transpose(2, 0, 1)                       # [896][7][26]
        assert np.array_equal(g, ovals), (name, b, np.argwhere(g != ovals)[:5])
        nfail += int((~cell_ok).sum())
        nflat_cell += int(flat[SLOT_CELL].all(axis=1).sum())
    print(f"{name}: {nfail} cells fall back, {nflat_cell} flat in every field, of "
          f"{len(rows) * NS}; values and verdicts bit for bit", flush=True)
    assert nfail > 0 or name == "leaf16"


# -- tolerance: networks with every weight non-zero -----------------------------

def _random_network(seed=13):
    return (np.random.default_rng(seed).normal(size=8090) * 0.3).astype(np.float32)


def _compare_tolerant(case, params, val, ok, y):
    """Element-wise comparison with the bounds of the module docstring;
    returns a summary dict."""
    W3 = np.abs(params[6400:8064].astype(np.float64)).max()
    rows = _oracle_rows(case, params)
    dy_all, nrow, ncell, flag_diff, flips, nline = [], 0, 0, 0, 0, 0
    field_err = np.zeros(7)
    field_max = np.zeros(7)
    for b, (yo, oval, rok, flat, sig, qc) in rows.items():
        sc = SLOT_CELL
        fl = flat[sc]                                       # [896][7]
        yg = y[b].transpose(1, 0, 2)                        # [896][7][26]
        yo_s = yo[sc]
        nf = ~fl
        dy = np.abs(yg - yo_s)                              # [896][7][26]
        dy_row = np.where(nf[..., None], dy, 0.0).max(axis=2)
        # raw outputs: every element within 2^-5 (1 + |y|) (a few bfloat16
        # flips, each ~|W3| 2^-8 |a|); the bulk far tighter
        lim = 2.0 ** -5 * (1.0 + np.abs(yo_s)) * max(1.0, W3 / 0.3)
        assert np.all(dy[nf] <= lim[nf]), (case.name, b, float(dy[nf].max()))
        dy_all.append(dy[nf].ravel())
        nrow += int(nf.sum())
        # verdicts
        cell_ok = rok[sc].all(axis=1)
        flag_diff += int((cell_ok != ok[b].astype(bool)).sum())
        ncell += NS
        # values on cells both sides pass
        both = cell_ok & ok[b].astype(bool)
        g = val[b].transpose(2, 0, 1)[both]                 # [m][7][26]
        o = oval[sc][both]
        s = sig[sc][both]
        q = qc[sc][both]
        dmax = dy_row[both]
        # (+ the two sides' binary32 roundings of offsets up to 2 sigma)
        bound = 2.0 * s * dmax + 2.0 ** -20 * s + 8.0 * np.spacing(np.maximum(np.abs(q), s))   # [m][7]
        err = np.abs(g - o)
        bad = err > bound[..., None]
        if bad.any():
            # lines one side flattened (both ends q_c) while the other did not,
            # with an end within the bound of q_c
            for m, f, d in zip(*np.nonzero(bad)):
                ln = np.nonzero((LINES == d).any(axis=1))[0][0]
                pp, mm = LINES[ln]
                qf = q[m, f]
                gflat = g[m, f, pp] == qf and g[m, f, mm] == qf
                oflat = o[m, f, pp] == qf and o[m, f, mm] == qf
                other = o[m, f] if gflat else g[m, f]
                near = min(abs(other[pp] - qf), abs(other[mm] - qf)) <= bound[m, f] + 1e-300
                assert gflat != oflat and near, (case.name, b, m, f, d, err[m, f, d], bound[m, f])
                flips += 1
        nline += int(both.sum()) * 7 * 13
        ok_err = np.where(bad, 0.0, err)
        field_err = np.maximum(field_err, ok_err.max(axis=(0, 2)) if ok_err.size else 0.0)
        field_max = np.maximum(field_max, np.abs(o).max(axis=(0, 2)) if o.size else 0.0)
    dy_all = np.concatenate(dy_all) if dy_all else np.zeros(1)
    # most rows see no bfloat16 flip at all: their outputs differ by FP32
    # rounding only
    assert np.median(dy_all) <= 1e-4, (case.name, float(np.median(dy_all)))
    return dict(rows=nrow, dy_max=float(dy_all.max()), dy_p999=float(np.quantile(dy_all, 0.999)),
                dy_median=float(np.median(dy_all)), cells=ncell, flag_diff=flag_diff,
                flips=flips // 2, lines=nline,
                field_rel=(field_err / np.maximum(field_max, 1e-300)))


@pytest.mark.parametrize("name", ["amr32", "polytrope", "leaf16"])
def test_random_network_values_elementwise(torch, name):
    case = _case(name)
    p = _random_network()
    print(f"case: pre-pass values, random network, {name}, {len(case.blocks)} blocks", flush=True)
    val, ok, y = _gpu_values(torch, case, p, want_y=True)
    r = _compare_tolerant(case, p, val, ok, y)
    print(f"{name}: {r['rows']} non-flat rows, |dy| median {r['dy_median']:.2e} p99.9 {r['dy_p999']:.2e} "
          f"max {r['dy_max']:.2e}; verdicts differ on {r['flag_diff']} of {r['cells']} cells; "
          f"{r['flips']} flattening flips of {r['lines']} lines; per-field rel "
          f"{np.array2string(r['field_rel'], precision=2)}", flush=True)
    assert r["flag_diff"] <= max(2, 0.005 * r["cells"])
    assert r["flips"] <= max(2, 0.001 * r["lines"])


@pytest.fixture(scope="module")
def trained(torch):
    from test_gpu_mlp import _quick_params
    print("case: quick training (2^17 pairs, 3 epochs)", flush=True)
    return _quick_params(torch)


def test_trained_network_values_elementwise_polytrope(torch, trained):
    case = _case("polytrope")
    print(f"case: pre-pass values, trained network, polytrope, {len(case.blocks)} blocks", flush=True)
    val, ok, y = _gpu_values(torch, case, trained, want_y=True)
    r = _compare_tolerant(case, trained, val, ok, y)
    print(f"polytrope/trained: {r['rows']} non-flat rows, |dy| median {r['dy_median']:.2e} "
          f"p99.9 {r['dy_p999']:.2e} max {r['dy_max']:.2e}; verdicts differ on {r['flag_diff']} of "
          f"{r['cells']} cells; {r['flips']} flattening flips; per-field rel "
          f"{np.array2string(r['field_rel'], precision=2)}", flush=True)
    assert r["flag_diff"] <= max(2, 0.005 * r["cells"])
    assert r["flips"] <= max(2, 0.001 * r["lines"])


# -- the learned stage ---------------------------------------------------------

@pytest.mark.parametrize("name", ["amr32", "polytrope"])
def test_constant_network_learned_stages_parity(torch, name):
    """Both stages of a learned step with the constant-output network: the
    GPU's values equal the oracle's bit for bit, so the stage results must
    meet the FP64 parity bound (per field and per element)."""
    from paper_2107_10987_amd.hydro import Hydro
    case = _case(name)
    p = _constant_network()
    ora = case.ora
    if name == "polytrope":
        # a contiguous Morton range across the star's edge
        l0 = int(case.edge_leaves[len(case.edge_leaves) // 2]) - 24
        l0 = min(max(l0, 0), case.tree.n - 48)
        l1 = l0 + 48
    else:
        l0, l1 = 0, case.tree.n
    print(f"case: learned stages 1 and 2, constant-output network, {name}, leaves [{l0}, {l1})", flush=True)
    hy = Hydro(max_leaves=case.tree.n, learned=True, schedule="column")
    try:
        hy.mlp_load(p)
        g = hy.grid(case.tree, torch.tensor(case.U, device="cuda"), case.omega, 5.0 / 3.0)
        a = hy.signal_speed(g).cpu().numpy()
        dt = float(0.4 * np.min(case.tree.dx / a))
        U1 = torch.empty_like(g.U)
        am = torch.empty(case.tree.n, dtype=torch.float64, device="cuda")
        hy.stage(g, 1, dt, g.U, g.U, U1, am)
        U1h = U1.cpu().numpy()
        am1 = am.cpu().numpy()
        U2 = torch.empty_like(g.U)
        hy.stage(g, 2, dt, U1, g.U, U2, am)
        U2h = U2.cpu().numpy()
        cells, fb = hy.mlp_stats()
    finally:
        hy.close()
    # (the returned arrays cover leaves [l0, l1))
    o1, oa1, ofb1 = ora.stage_learned(p, 1, dt, case.U, l0=l0, l1=l1)
    assert np.abs(am1[l0:l1] - oa1).max() <= 1e-12 * oa1.max()
    parity.check(U1h[l0:l1], o1, ora, case.U, label=f"{name} stage 1", l0=l0, l1=l1)
    # stage 2 needs the stage-1 state of every leaf (ghosts): whole meshes only
    if l0 == 0 and l1 == case.tree.n:
        o2, oa2, ofb2 = ora.stage_learned(p, 2, dt, o1, case.U)
        parity.check(U2h, o2, ora, o1, extra=(case.U,), label=f"{name} stage 2")
        assert np.abs(am.cpu().numpy() - oa2).max() <= 1e-12 * oa2.max()   # stage 2's own speeds
    print(f"{name}: fallback cells gpu {fb} of {cells} (both stages, all leaves), "
          f"oracle stage 1 on the range {int(ofb1.sum())}", flush=True)
    assert np.isfinite(U2h).all()


def test_trained_network_learned_stage_polytrope(torch, trained):
    """Stage 1 of a learned step with the trained network on a Morton range
    across the star's edge: the network's outputs differ between the sides
    by FP32 rounding and rare bfloat16 flips (median |dy| ~1e-8), the point
    values by at most 2 sigma |dy|, so each cell's update differs by at most
    dt/dx times such value differences in the fluxes; per field,
    max |g - o| / max |o_f| <= 1e-5 (CFL 0.4 times the largest value error,
    ~1e-4 of a field's range, per the values test above)."""
    from paper_2107_10987_amd.hydro import Hydro
    case = _case("polytrope")
    l0 = int(case.edge_leaves[len(case.edge_leaves) // 2]) - 24
    l0 = min(max(l0, 0), case.tree.n - 48)
    l1 = l0 + 48
    print(f"case: learned stage 1, trained network, polytrope, leaves [{l0}, {l1})", flush=True)
    hy = Hydro(max_leaves=case.tree.n, learned=True, schedule="column")
    try:
        hy.mlp_load(trained)
        g = hy.grid(case.tree, torch.tensor(case.U, device="cuda"), case.omega, 5.0 / 3.0)
        a = hy.signal_speed(g).cpu().numpy()
        dt = float(0.4 * np.min(case.tree.dx / a))
        U1 = torch.empty_like(g.U)
        am = torch.empty(case.tree.n, dtype=torch.float64, device="cuda")
        hy.stage(g, 1, dt, g.U, g.U, U1, am)
        U1h = U1.cpu().numpy()[l0:l1]
        am1 = am.cpu().numpy()[l0:l1]
    finally:
        hy.close()
    o1, oa1, ofb1 = case.ora.stage_learned(trained, 1, dt, case.U, l0=l0, l1=l1)
    # per field against the field's largest value; the momenta against the
    # largest momentum component (the star rotates about z, so its z momentum
    # is only what one stage of pressure forces gives it)
    g3, o3 = U1h.reshape(48, 7, -1), o1.reshape(48, 7, -1)
    scale = np.abs(o3).max(axis=(0, 2))
    scale[1:4] = scale[1:4].max()
    fe = np.abs(g3 - o3).max(axis=(0, 2)) / scale
    da = np.abs(am1 - oa1).max() / oa1.max()
    print(f"trained stage 1: per-field {np.array2string(fe, precision=2)}; signal speed {da:.2e}; "
          f"oracle fallback cells {int(ofb1.sum())}", flush=True)
    assert np.all(fe <= 1e-5), fe
    assert da <= 1e-5
