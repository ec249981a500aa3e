"""Pins of the oracle's closure pieces: bfloat16 rounding, network gradients, Adam, spectral
truncation, and the column feature / correction definitions.

* bfloat16 rounding: exact representable values and ties to even, and agreement with torch's
  own CPU conversion.
* Gradients of the FP64 network (no rounding) against central differences of the loss.
* Adam: the first bias-corrected step moves every weight by lr * g / (|g| + eps).
* Truncation: a field whose spectrum lies in the coarse set, evaluated at the coarse nodes term
  by term from the fine coefficients (Eq. expansion), equals the coarse backward transform of
  the truncated coefficients.
* Features, targets and corrections on single coefficients placed by hand.
"""
import numpy as np
import pytest

from oracle import closure as oc
from oracle.basis import pbar
from oracle.grid import Grid
from oracle.transform import Tables, backward


def test_bf16_exact_values_and_ties():
    one = 1.0
    ulp = 2.0 ** -7
    vals = np.array([one, one + ulp, one + 0.5 * ulp, one + 1.5 * ulp, -(one + 0.5 * ulp), 3.0 * 2.0 ** -130,
                     one + 0.5 * ulp + 2.0 ** -20, 0.0, -0.0])
    want = np.array([one, one + ulp, one, one + 2 * ulp, -one, 3.0 * 2.0 ** -130, one + ulp, 0.0, 0.0])
    np.testing.assert_array_equal(oc.bf16_round(vals), want)


def test_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    v = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oc.bf16_round(v.astype(np.float64)), ref)


def _tiny_net(seed, nin=7, h=6, nout=4, nb=5):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((nb, nin))
    t = rng.standard_normal((nb, nout))
    W1 = rng.standard_normal((h, nin)) * 0.5
    b1 = rng.standard_normal(h) * 0.1
    W2 = rng.standard_normal((h, h)) * 0.5
    b2 = rng.standard_normal(h) * 0.1
    W3 = rng.standard_normal((nout, h)) * 0.5
    b3 = rng.standard_normal(nout) * 0.1
    return x, t, dict(W1=W1, b1=b1, W2=W2, b2=b2, W3=W3, b3=b3)


def test_gradients_match_central_differences():
    x, t, P = _tiny_net(11)
    names = ("W1", "b1", "W2", "b2", "W3", "b3")
    _, g = oc.loss_and_grads(x, t, *[P[k] for k in names], rounding=False)
    h = 1e-6
    for k in names:
        fd = np.zeros_like(P[k])
        it = np.nditer(P[k], flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            Pp = {q: v.copy() for q, v in P.items()}
            Pm = {q: v.copy() for q, v in P.items()}
            Pp[k][i] += h
            Pm[k][i] -= h
            lp, _ = oc.loss_and_grads(x, t, *[Pp[q] for q in names], rounding=False)
            lm, _ = oc.loss_and_grads(x, t, *[Pm[q] for q in names], rounding=False)
            fd[i] = (lp - lm) / (2 * h)
        err = np.linalg.norm(g[k] - fd) / np.linalg.norm(fd)
        assert err < 1e-6, (k, err)


def test_gradient_of_a_wrong_sign_fails_the_pin():
    # the same check on a planted mistake (sign of the tanh derivative) must fail
    x, t, P = _tiny_net(12)
    names = ("W1", "b1", "W2", "b2", "W3", "b3")
    _, g = oc.loss_and_grads(x, t, *[P[k] for k in names], rounding=False)
    h = 1e-6
    Pp = {q: v.copy() for q, v in P.items()}
    Pm = {q: v.copy() for q, v in P.items()}
    Pp["b1"][0] += h
    Pm["b1"][0] -= h
    lp, _ = oc.loss_and_grads(x, t, *[Pp[q] for q in names], rounding=False)
    lm, _ = oc.loss_and_grads(x, t, *[Pm[q] for q in names], rounding=False)
    fd = (lp - lm) / (2 * h)
    f = oc.forward(x, *[P[k] for k in names], rounding=False)
    dy = 2 * (f["y"] - t) / f["y"].size
    dz2 = (dy @ P["W3"]) * (1 - f["h2"] ** 2)
    wrong = ((dz2 @ P["W2"]) * (1 + f["h1"] ** 2)).sum(0)[0]
    assert abs(g["b1"][0] - fd) < 1e-8 * max(1.0, abs(fd))
    assert abs(wrong - fd) > 1e-4 * abs(fd)


def test_rounding_points_change_results_by_bf16_amounts():
    x, t, P = _tiny_net(13, nin=40, h=32, nout=16, nb=64)
    names = ("W1", "b1", "W2", "b2", "W3", "b3")
    l0, g0 = oc.loss_and_grads(x, t, *[P[k] for k in names], rounding=False)
    l1, g1 = oc.loss_and_grads(x, t, *[P[k] for k in names], rounding=True)
    for k in names:
        rel = np.linalg.norm(g1[k] - g0[k]) / np.linalg.norm(g0[k])
        assert 1e-5 < rel < 5e-2, (k, rel)
    assert abs(l1 - l0) / l0 < 5e-2


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p = rng.standard_normal(100)
    g = rng.standard_normal(100) * np.exp(rng.uniform(-6, 2, 100))
    lr = 1e-3
    p1, m1, v1 = oc.adam_step(p, g, np.zeros(100), np.zeros(100), 1, lr)
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # a constant gradient keeps the bias-corrected ratio: the second step is the same move
    p2, _, _ = oc.adam_step(p1, g, m1, v1, 2, lr)
    np.testing.assert_allclose(p2 - p1, p1 - p, rtol=1e-9, atol=1e-18)


def _expansion_at(S, M, nrc, nz, lz, x, phi, z):
    """Eq. expansion summed term by term from coefficients S[m, n, slot] of an N_z-slot axis."""
    kv = np.fft.fftfreq(nz, d=1.0 / nz).round().astype(int)
    out = np.zeros((len(z), len(x), len(phi)))
    for m in range(M):
        P = pbar(m, nrc, np.asarray(x, dtype=np.longdouble)).astype(np.float64)
        for s in range(nz):
            k = kv[s]
            for n in range(m, nrc):
                c = S[m, n, s]
                if c == 0:
                    continue
                e = np.exp(1j * m * phi[None, None, :] + 2j * np.pi * k * z[:, None, None] / lz)
                term = c * P[n][None, :, None] * e
                out += (term.real if m == 0 else 2 * term.real)
    return out


def test_truncation_is_exact_for_coarse_band_limited_fields():
    gf = Grid(nr=10, nphi=8, nz=8, ell=1.3, lz=5.0)
    gc = Grid(nr=6, nphi=6, nz=6, ell=1.3, lz=5.0)
    rng = np.random.default_rng(8)
    kvf = gf.kvals()
    S = np.zeros((gf.M, gf.nrc, gf.nz), dtype=np.complex128)
    for m in range(gc.M):
        for s, k in enumerate(kvf):
            if abs(k) < gc.nzc and not (gc.nz % 2 == 0 and k == -(gc.nz // 2)):
                for n in range(m, gc.nrc):
                    S[m, n, s] = rng.standard_normal() + 1j * rng.standard_normal()
    # a real field: m = 0 Hermitian in k
    slot = {int(k): i for i, k in enumerate(kvf)}
    for s, k in enumerate(kvf):
        if k < 0 and S[0, :, s].any():
            S[0, :, s] = np.conj(S[0, :, slot[-k]])
    S[0, :, slot[0]] = S[0, :, slot[0]].real
    Sc = oc.truncate(S, gf.nzc, gc.M, gc.nrc, gc.nz, gc.nzc)
    direct = _expansion_at(S, gf.M, gf.nrc, gf.nz, gf.lz, gc.x, gc.phi, gc.z)
    via = backward(Sc, gc, Tables(gc))
    np.testing.assert_allclose(via, direct, rtol=0, atol=1e-12 * np.abs(direct).max())
    # and back: zero extension restores the fine coefficients
    Sf = oc.truncate(Sc, gc.nzc, gf.M, gf.nrc, gf.nz, gf.nzc)
    np.testing.assert_array_equal(Sf, S)


def test_features_targets_and_correction_on_single_coefficients():
    M, nrc, nz, nzc = 4, 6, 8, 4   # kept k: 0, 1, 2, 3, -3, -2, -1
    cols, slots = oc.columns(M, nz, nzc)
    assert slots == [0, 1, 2, 3, 5, 6, 7] and len(cols) == 28
    Sp = np.zeros((M, nrc, nz), dtype=np.complex128)
    Sc = np.zeros_like(Sp)
    Sp[2, 5, 6] = 1.5 - 2.0j      # m = 2, n = 5, k = -2 (slot 6)
    Sc[1, 3, 1] = 0.25 + 0.5j     # m = 1, n = 3, k = 1
    X = oc.features(Sp, Sc, nzc)
    c1 = cols.index((2, 6))
    c2 = cols.index((1, 1))
    nz_entries = {(r, j) for r, j in zip(*np.nonzero(X[:, :256]))}
    assert nz_entries == {(c1, 5), (c1, 69), (c2, 128 + 3), (c2, 192 + 3)}
    assert X[c1, 5] == 1.5 and X[c1, 69] == -2.0 and X[c2, 131] == 0.25 and X[c2, 195] == 0.5
    assert X[c1, 256] == np.float32(0.5) and X[c1, 257] == np.float32(-2.0 / 3.0)
    Y = oc.targets(Sp, Sc, Sc, Sp, nzc)
    assert Y[c1, 5] == 1.5 and Y[c2, 131] == 0.25 and Y[c1, 128 + 5] == -1.5 and Y[c2, 3] == -0.25
    # correction: a single output lands on its coefficient; m = 0 is made Hermitian
    Yc = np.zeros((len(cols), 256), dtype=np.float32)
    Yc[c1, 64 + 5] = 3.0
    c0 = cols.index((0, 1))
    Yc[c0, 2] = 1.0
    Yc[c0, 64 + 2] = 2.0
    Cp, Cc = oc.correction(Yc, M, nrc, nz, nzc)
    assert Cp[2, 5, 6] == 3.0j and not Cc.any()
    assert Cp[0, 2, 1] == 0.5 + 1.0j and Cp[0, 2, 7] == 0.5 - 1.0j
    assert np.count_nonzero(Cp) == 3


def test_judge_rules():
    R = np.ones((2, 3, 4), dtype=np.complex128)
    C = 0.1 * R
    assert oc.judge(C, C, R, R, 0.2)
    assert not oc.judge(C, C, R, R, 0.05)
    assert not oc.judge(C * np.nan, C, R, R, 10.0)
    assert oc.judge(0 * C, 0 * C, R, R, 0.0)
    # reference judge: a correction towards the finer-grid term is kept, one away from it dropped
    A = R + 0.2 * R
    assert oc.judge(C, C, R, R, 10.0, ref=(A, A))
    assert not oc.judge(-C, -C, R, R, 10.0, ref=(A, A))
    assert oc.judge(0 * C, 0 * C, R, R, 10.0, ref=(R, R))          # equal distances: kept
    assert not oc.judge(C, C, R, R, 10.0, ref=(R, R))
    assert not oc.judge(C, C, R, R, 10.0, ref=(A * np.nan, A))
