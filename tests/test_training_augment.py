"""The training pairs' augmentation by the cube's symmetries and sign flips
(CPU, torch on the host).  A symmetry R applied to a whole padded block --
cells moved to R c about the block centre, momentum components permuted and
sign-changed as a vector -- must turn the oracle's pair (features, plain-PPM
targets) of cell c and field f into the oracle's pair of cell R c and field
f' of the transformed block; augment_rows must produce exactly that from the
original row.  Same for the sign flip of a field."""
import numpy as np
import pytest

from paper_2107_10987_amd.learned import augment_rows, symmetry_tables
from paper_2107_10987_amd.workloads import blast_single_leaf


def _rows(oracle_mod, P, cells):
    V = oracle_mod.reconstruct_values(P)
    X, T, keys = [], [], []
    for (i, j, k) in cells:
        for f in range(7):
            nb, s, x = oracle_mod.mlp_features(P, i, j, k, f)
            if x is None:
                continue
            c = (k + 1) * 100 + (j + 1) * 10 + (i + 1)
            X.append(x.astype(np.float32))
            T.append(((V[c, :, f] - nb[13]) * (1.0 / s)).astype(np.float32))
            keys.append((i, j, k, f))
    return np.array(X), np.array(T), keys


def _transform_block(P, perm, sg):
    """P' with P'[f'][R c] = e P[f][c], R about the block centre (cells
    -3..10, centre 3.5)."""
    Q = np.empty_like(P)
    idx = np.arange(14)
    for f in range(7):
        fp, e = f, 1.0
        if 1 <= f <= 3:
            a = f - 1
            fp, e = 1 + perm[a], float(sg[a])
        src = P[f]                                     # [k][j][i]
        # P'[R c] = e P[c]: for each target index along axis perm[a] take the
        # source index along axis a, reflected if sg[a] < 0
        out = np.empty_like(src)
        for kk in idx:
            for jj in idx:
                for ii in idx:
                    tgt = [ii, jj, kk]
                    c = [0, 0, 0]
                    for a in range(3):
                        t = tgt[perm[a]]
                        c[a] = t if sg[a] > 0 else 13 - t
                    out[kk, jj, ii] = src[c[2], c[1], c[0]]
        Q[fp] = e * out
    return Q


def test_symmetry_tables_form_the_cube_group():
    gx, gt, fmap, fsign = symmetry_tables()
    assert gx.shape == (48, 27) and gt.shape == (48, 26)
    assert len({tuple(r) for r in gx}) == 48
    assert np.all(gx[:, 13] == 13)
    for r in gx:
        assert sorted(r) == list(range(27))


@pytest.mark.parametrize("k", [0, 7, 13, 29, 47])
def test_augmented_rows_are_the_transformed_blocks_rows(oracle_mod, k):
    torch = pytest.importorskip("torch")
    import itertools
    w = blast_single_leaf()
    o = oracle_mod.Oracle(w.tree, w.gamma, w.omega)
    U, _ = o.step(o.dt(w.U), w.U)
    rng = np.random.default_rng(3)
    U = U.copy()
    U[:, 1:4] += rng.normal(size=U[:, 1:4].shape) * 1e-3      # momenta of both signs
    P = o.padded(U)[0]
    perms = list(itertools.permutations(range(3)))
    perm, bits = perms[k // 8], k % 8
    sg = [-1 if (bits >> a) & 1 else 1 for a in range(3)]
    cells = [(2, 3, 4), (3, 3, 3), (4, 4, 3), (0, 5, 7), (6, 1, 2)]
    X, T, keys = _rows(oracle_mod, P, cells)
    Xt, Tt = (torch.tensor(a) for a in (X, T))
    for sign in (1, -1):
        Xa, Ta = augment_rows(torch, Xt, Tt, np.arange(len(keys)), np.full(len(keys), k),
                              np.full(len(keys), sign))
        Q = sign * _transform_block(P, perm, sg)
        Vq = oracle_mod.reconstruct_values(Q)
        for r, (i, j, kk, f) in enumerate(keys):
            c = [i, j, kk]
            rc = [0, 0, 0]
            for a in range(3):
                rc[perm[a]] = c[a] if sg[a] > 0 else 7 - c[a]
            fp = 1 + perm[f - 1] if 1 <= f <= 3 else f
            nb, s, x = oracle_mod.mlp_features(Q, rc[0], rc[1], rc[2], fp)
            assert x is not None
            assert np.array_equal(Xa[r].numpy(), x.astype(np.float32)), (k, sign, r)
            cq = (rc[2] + 1) * 100 + (rc[1] + 1) * 10 + (rc[0] + 1)
            t = ((Vq[cq, :, fp] - nb[13]) * (1.0 / s)).astype(np.float32)
            # a line evaluated in the other orientation may round its ends
            # differently by an ulp of the FP64 values
            assert np.allclose(Ta[r].numpy(), t, rtol=0, atol=1e-6), (k, sign, r)
