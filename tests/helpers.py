"""Shared pieces of the GPU tests: progress lines and the gradient bar."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def grad_compare(name, got, ref, rel=1e-3):
    """Per tensor: |got - ref| <= rel |ref| (2-norm), and at most 0.1% of the
    elements outside 2e-3 (|ref| + 1e-2 max|ref|)."""
    got = np.asarray(got, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    nr = np.linalg.norm(ref)
    err = np.linalg.norm(got - ref)
    say(f"  grad {name}: |ref| {nr:.3e} rel err {err / max(nr, 1e-30):.2e}")
    if nr == 0:
        assert np.abs(got).max(initial=0.0) <= 1e-6, name
        return
    assert err <= rel * nr, name
    m = np.abs(ref).max()
    bad = np.abs(got - ref) > 2e-3 * (np.abs(ref) + 1e-2 * m)
    assert bad.mean() <= 1e-3, (name, int(bad.sum()))


def packed_loss_oracle(oracle, renders, targets, lambda_t=0.1, k=20.0):
    """The loss of several images packed together from the oracle's per-image
    loss: the means run over all pixels, so image c's loss and gradients are
    weighted by its share of the pixels. Returns (L, [(gi, gt, gm)] per image)."""
    n_all = sum(t.shape[1] * t.shape[2] for t in targets)
    L = 0.0
    ups = []
    for o, tgt in zip(renders, targets):
        w = tgt.shape[1] * tgt.shape[2] / n_all
        Lc, gi, gt, gm = oracle.loss(o["image"], o["final_T"], o["mesh_rgb"], o["tri_id"], tgt,
                                     lambda_t=lambda_t, k=k)
        L += w * Lc
        ups.append((gi * w, gt * w, gm * w))
    return L, ups


AMB_ALPHA, AMB_T, AMB_PROJ, AMB_MESH, AMB_MANY = 1, 2, 4, 16, 32


def check_pixels(view, orc, img_tol=1e-4):
    """Every pixel of a GPU view (image, T, mesh_rgb, mesh_depth, tri_id,
    n_contrib, n_blended, n_processed) against an oracle render made with
    alts=True. Pixels whose only ambiguity is an alpha-skip or T-stop decision
    inside the FP32 slack must equal one of the oracle's outcomes of the paths
    through those decisions (colour and T within img_tol, counts exact); the
    rest must equal the oracle's FP64 outcome. Pixels near a projection or
    mesh-depth rounding boundary, or with more paths than the oracle keeps,
    are left out of the blend checks. Returns (left out, checked by paths)."""
    im, T, mr, md, tri, nc, nb, npro = view
    amb = orc["amb"]
    hard = (amb & (AMB_PROJ | AMB_MESH | AMB_MANY)) != 0
    soft = ((amb & (AMB_ALPHA | AMB_T)) != 0) & ~hard
    good = amb == 0
    np.testing.assert_array_equal(tri, orc["tri_id"])
    mesh_ok = (amb & AMB_MESH) == 0
    np.testing.assert_array_equal(md[mesh_ok], orc["mesh_depth"][mesh_ok])
    np.testing.assert_allclose(mr, orc["mesh_rgb"], atol=1e-5)
    d_img = np.abs(im - orc["image"])[:, good]
    d_T = np.abs(T - orc["final_T"])[good]
    assert d_img.size == 0 or d_img.max() <= img_tol, d_img.max()
    assert d_T.size == 0 or d_T.max() <= img_tol, d_T.max()
    np.testing.assert_array_equal(nc[good], orc["n_contrib"][good])
    np.testing.assert_array_equal(nb[good], orc["n_blended"][good])
    np.testing.assert_array_equal(npro[good], orc["n_processed"][good])
    if soft.any():
        ys, xs = np.nonzero(soft)
        al = orc["alts"][ys, xs]                     # [k, MAX_ALT, 7]
        na = orc["n_alt"][ys, xs]
        gv = np.column_stack([im[:, ys, xs].T, T[ys, xs], nc[ys, xs], nb[ys, xs], npro[ys, xs]])
        close = (np.abs(al[..., :4] - gv[:, None, :4]) <= img_tol).all(-1)
        same = (al[..., 4:] == gv[:, None, 4:]).all(-1)
        valid = np.arange(al.shape[1])[None, :] < na[:, None]
        ok = (close & same & valid).any(1)
        assert ok.all(), f"{int((~ok).sum())} ambiguous pixels match none of the oracle's paths"
    return int(hard.sum()), int(soft.sum())
