"""The learned closure on the GPU: parity with the oracle, the judge, and time integration.

* Spectral truncation between grids: bit-exact against the oracle.
* Column features and targets: bit-exact against the oracle.
* Network forward, loss and gradients: against the oracle's FP64 network with the same bfloat16
  rounding points (normwise <= 1e-3, the bound set by bfloat16 rounding ties); Adam against the
  oracle's update from the GPU's own gradients.
* Judge: forced fallbacks (beta = 0, non-finite weights) leave the coarse term unchanged; an
  accepted correction equals the oracle's features -> network -> Hermitian correction.
* mlg_tp_advance equals the same sequence of single entry points, bit for bit, with and without
  the closure, and across split calls.
"""
import numpy as np
import pytest

import synth
from helpers import from_lib, rel, to_lib
from oracle import closure as oc
from oracle.grid import Grid

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-3


def _say(*a):
    print(*a, flush=True)


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_18026_amd as m
    return m


def _dev(S):
    return torch.from_numpy(to_lib(S)).cuda()


def test_truncate_parity_and_zero_extension():
    m = _gpu()
    _say("truncate parity")
    gf = Grid(24, 16, 16, 1.2, lz=5.0)
    gc = Grid(12, 8, 10, 1.2, lz=5.0)
    fine = m.Plan(24, 16, 16, 1.2, 5.0)
    coarse = m.Plan(12, 8, 10, 1.2, 5.0)
    S = synth.geometric_spectrum(gf.M, gf.nrc, gf.nz, gf.nzc, seed=21)
    out = coarse.empty_spec()
    fine.truncate_to(coarse, _dev(S), out)
    torch.cuda.synchronize()
    ref = oc.truncate(S, gf.nzc, gc.M, gc.nrc, gc.nz, gc.nzc)
    np.testing.assert_array_equal(from_lib(out.cpu().numpy(), gc.M, gc.nrc), ref)
    back = fine.empty_spec()
    coarse.truncate_to(fine, out, back)
    torch.cuda.synchronize()
    ref2 = oc.truncate(ref, gc.nzc, gf.M, gf.nrc, gf.nz, gf.nzc)
    np.testing.assert_array_equal(from_lib(back.cpu().numpy(), gf.M, gf.nrc), ref2)
    other = m.Plan(12, 8, 10, 1.3, 5.0)
    with pytest.raises(m.MlgError):
        fine.truncate_to(other, _dev(S), other.empty_spec())


def _coarse(m, nr=16, nphi=12, nz=10, ell=0.9, lz=4.0, max_batch=512, beta=1.0):
    g = Grid(nr, nphi, nz, ell, lz=lz)
    plan = m.Plan(nr, nphi, nz, ell, lz)
    return g, plan, m.Closure(plan, max_batch=max_batch, beta=beta)


def test_features_and_targets_bit_exact():
    m = _gpu()
    _say("features/targets parity")
    g, plan, cl = _coarse(m)
    sp = synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=31, a=0.8)
    sc = synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=32, a=0.8)
    X = torch.empty((cl.ncols, 258), dtype=torch.float32, device="cuda")
    cl.features(_dev(sp), _dev(sc), X)
    torch.cuda.synchronize()
    ref = oc.features(sp, sc, g.nzc)
    assert cl.ncols == ref.shape[0]
    np.testing.assert_array_equal(X.cpu().numpy(), ref)
    R = [synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=40 + i, a=0.8) for i in range(4)]
    Y = torch.empty((cl.ncols, 256), dtype=torch.float32, device="cuda")
    cl.targets(*[_dev(r) for r in R], Y)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Y.cpu().numpy(), oc.targets(*R, g.nzc))


def _random_problem(seed, nb, count=None):
    r = np.random.default_rng(seed)
    count = count or nb
    params = synth.closure_init(seed, last_gain=1.0)
    params[256 * 258:256 * 258 + 256] = r.standard_normal(256).astype(np.float32) * 0.1   # b1
    xs = np.exp(r.uniform(-1, 1, 258)).astype(np.float32)
    ys = np.exp(r.uniform(-1, 1, 256)).astype(np.float32)
    X = r.standard_normal((count, 258)).astype(np.float32)
    Y = r.standard_normal((count, 256)).astype(np.float32)
    return params, xs, ys, X, Y


def _oracle_inputs(params, xs, ys, X, Y):
    # the scaled inputs and targets are formed in float32 on both sides
    xt = (X * xs[None, :]).astype(np.float64)
    tt = (Y / ys[None, :]).astype(np.float64)
    return xt, tt, oc.network_params(params)


@pytest.mark.parametrize("nb", [1, 300, 2048])
def test_forward_parity(nb):
    m = _gpu()
    _say("closure forward parity nb", nb)
    g, plan, cl = _coarse(m, max_batch=2048)
    params, xs, ys, X, Y = _random_problem(50 + nb, nb)
    cl.set_params(params)
    cl.set_scales(xs, ys)
    y = torch.empty((nb, 256), dtype=torch.float32, device="cuda")
    cl.forward(torch.from_numpy(X).cuda(), y)
    torch.cuda.synchronize()
    xt, tt, P = _oracle_inputs(params, xs, ys, X, Y)
    ref = oc.forward(xt, *P)["y"] * ys[None, :]
    err = rel(y.cpu().numpy(), ref)
    _say("  forward rel", err)
    assert err < TOL


@pytest.mark.parametrize("nb,count,indexed", [(300, 300, False), (4096, 6000, True), (65, 100, True)])
def test_gradient_and_adam_parity(nb, count, indexed):
    m = _gpu()
    _say("closure gradient parity", nb, count, indexed)
    g, plan, cl = _coarse(m, max_batch=4096)
    params, xs, ys, X, Y = _random_problem(70 + nb, nb, count)
    cl.set_params(params)
    cl.set_scales(xs, ys)
    idx = None
    rows = np.arange(nb)
    if indexed:
        rows = synth.batch_indices(count, nb, 1, seed=nb)[0]
        idx = torch.from_numpy(rows).cuda()
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    loss = cl.train_step(Xd, Yd, idx, nb, 0.0, want_loss=True)
    g1 = cl.get_grads()
    np.testing.assert_array_equal(cl.get_params(), params)   # lr = 0 leaves the weights alone
    xt, tt, P = _oracle_inputs(params, xs, ys, X[rows], Y[rows])
    ref_loss, ref_g = oc.loss_and_grads(xt, tt, *P)
    assert abs(loss - ref_loss) / ref_loss < 1e-5, (loss, ref_loss)
    o = 0
    for name, sz in (("W1", 256 * 258), ("b1", 256), ("W2", 65536), ("b2", 256), ("W3", 65536), ("b3", 256)):
        err = rel(g1[o:o + sz], ref_g[name].reshape(-1))
        _say("  grad", name, err)
        assert err < TOL, (name, err)
        o += sz
    # a second step with a learning rate: Adam from the GPU's own gradients (step count 2)
    lr = 1e-3
    cl.train_step(Xd, Yd, idx, nb, lr)
    g2 = cl.get_grads()
    p2 = cl.get_params()
    mom = 0.1 * g1.astype(np.float64)
    vel = 0.001 * g1.astype(np.float64) ** 2
    ref_p, _, _ = oc.adam_step(params.astype(np.float64), g2.astype(np.float64), mom, vel, 2, lr)
    upd = rel(p2.astype(np.float64) - params, ref_p - params)
    _say("  adam update rel", upd)
    assert upd < 1e-4


def test_bad_batch_index_is_reported():
    m = _gpu()
    g, plan, cl = _coarse(m, max_batch=128)
    params, xs, ys, X, Y = _random_problem(90, 64)
    cl.set_params(params)
    idx = torch.arange(64, dtype=torch.int32, device="cuda")
    idx[5] = 64
    with pytest.raises(m.MlgError):
        cl.train_step(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), idx, 64, 1e-3, want_loss=True)
    # the flag is cleared: a valid call succeeds
    idx[5] = 3
    cl.train_step(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), idx, 64, 1e-3, want_loss=True)


def _state(g, seed):
    return (synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=seed, a=0.8, b=0.8, c=0.8),
            synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=seed + 1, a=0.8, b=0.8, c=0.8))


def test_judge_accepts_with_oracle_correction():
    m = _gpu()
    _say("closure judge / accepted correction")
    g, plan, cl = _coarse(m, beta=1e30)
    params, xs, ys, _, _ = _random_problem(91, 1)
    params *= 0.5
    cl.set_params(params)
    cl.set_scales(xs * 0.1, ys * 1e-3)
    sp, sc = _state(g, 60)
    rp, rc = _state(g, 62)
    a, b = _dev(rp), _dev(rc)
    fb = cl.infer(_dev(sp), _dev(sc), a, b, want_flag=True)
    assert fb == 0
    X = oc.features(sp, sc, g.nzc)
    xt = (X * (xs * 0.1)[None, :]).astype(np.float64)
    Yo = oc.forward(xt, *oc.network_params(params))["y"] * (ys * 1e-3)[None, :]
    Cp, Cc = oc.correction(Yo, g.M, g.nrc, g.nz, g.nzc)
    gp = from_lib(a.cpu().numpy(), g.M, g.nrc) - rp
    gc = from_lib(b.cpu().numpy(), g.M, g.nrc) - rc
    err = rel(np.concatenate([gp.ravel(), gc.ravel()]), np.concatenate([Cp.ravel(), Cc.ravel()]))
    _say("  applied correction rel", err)
    assert err < TOL
    # m = 0 stays Hermitian in k
    kv = g.kvals()
    slot = {int(k): i for i, k in enumerate(kv)}
    for i, k in enumerate(kv):
        if g.kmask()[i] and k > 0:
            np.testing.assert_allclose(gp[0, :, slot[-k]], np.conj(gp[0, :, i]), rtol=0, atol=1e-12)
    assert cl.stats() == (1, 0)


@pytest.mark.parametrize("case", ["zero_net_same_grid", "net_same_grid", "net_finer_grid"])
def test_reference_judge_decision(case):
    """The reference judge against the oracle's decision on the library's own terms: a network with
    zero output is always kept (equal distances), any other correction is dropped when the reference
    plan has the coarse grid (the reference term is then the plain term), and on a finer reference
    the decision follows ||A_c + C - Ar|| <= ||A_c - Ar||."""
    m = _gpu()
    _say("closure reference judge", case)
    g, plan, cl = _coarse(m, beta=1e30)
    params, xs, ys, _, _ = _random_problem(93, 1)
    if case == "zero_net_same_grid":
        params[:] = 0.0
    cl.set_params(params)
    cl.set_scales(xs * 0.1, ys * 1e-2)
    nr, nphi, nz = (16, 12, 10) if case != "net_finer_grid" else (24, 18, 16)
    ref = m.Plan(nr, nphi, nz, 0.9, 4.0, nrc=16, nphic=6, nzc=5)
    U = (0.0, 1.0, 0.0)
    cl.set_reference(ref, U)
    sp, sc = _state(g, 64)
    P, Cc = _dev(sp), _dev(sc)
    a, b = plan.empty_spec(), plan.empty_spec()
    plan.rhs_tp(P, Cc, a, b, U=U)
    a0, b0 = a.clone(), b.clone()
    # the oracle's decision from the library's terms: the plain term, the unjudged correction and
    # the reference term truncated back
    free = m.Closure(plan, max_batch=512, beta=1e30)
    free.set_params(params)
    free.set_scales(xs * 0.1, ys * 1e-2)
    ca, cb = a0.clone(), b0.clone()
    free.infer(P, Cc, ca, cb)
    qp, qc = ref.empty_spec(), ref.empty_spec()
    plan.truncate_to(ref, P, qp)
    plan.truncate_to(ref, Cc, qc)
    rp, rc = ref.empty_spec(), ref.empty_spec()
    ref.rhs_tp(qp, qc, rp, rc, U=U)
    tp, tc = plan.empty_spec(), plan.empty_spec()
    ref.truncate_to(plan, rp, tp)
    ref.truncate_to(plan, rc, tc)
    fb = cl.infer(P, Cc, a, b, want_flag=True)
    torch.cuda.synchronize()
    h = lambda t: from_lib(t.cpu().numpy(), g.M, g.nrc)
    R0p, R0c = h(a0), h(b0)
    keep = oc.judge(h(ca) - R0p, h(cb) - R0c, R0p, R0c, 1e30, ref=(h(tp), h(tc)))
    _say("  oracle keeps", keep, "library fallback", fb)
    assert fb == (0 if keep else 1)
    if case == "zero_net_same_grid":
        assert keep
    if case == "net_same_grid":
        assert not keep
    if keep:
        assert torch.equal(a, ca) and torch.equal(b, cb)
    else:
        assert torch.equal(a, a0) and torch.equal(b, b0)
    cl.set_reference(None)
    for x in (free, cl, ref, plan):
        x.close()


@pytest.mark.parametrize("mode", ["beta0", "nan"])
def test_forced_fallback_keeps_plain_term(mode):
    m = _gpu()
    _say("closure forced fallback", mode)
    g, plan, cl = _coarse(m, beta=0.0 if mode == "beta0" else 10.0)
    params, xs, ys, _, _ = _random_problem(92, 1)
    if mode == "nan":
        params[1000] = np.nan
    cl.set_params(params)
    sp, sc = _state(g, 70)
    rp, rc = _state(g, 72)
    a, b = _dev(rp), _dev(rc)
    a0, b0 = a.clone(), b.clone()
    assert cl.infer(_dev(sp), _dev(sc), a, b, want_flag=True) == 1
    assert torch.equal(a, a0) and torch.equal(b, b0)
    cl.infer(_dev(sp), _dev(sc), a, b)   # no flag requested: asynchronous
    assert cl.stats() == (2, 2)


def _manual(plan, psi, chi, n, U, closure=None):
    """Richardson start then AB-CN, through the single-step entry points."""
    def A(p, c):
        ap, ac = plan.empty_spec(), plan.empty_spec()
        plan.rhs_tp(p, c, ap, ac, U=U)
        if closure is not None:
            closure.infer(p, c, ap, ac)
        return ap, ac

    def febe(half, s, a):
        o = plan.empty_spec()
        plan.step_febe(half, s, a, o)
        return o

    A0 = A(psi, chi)
    full = [febe(0, s, a) for s, a in zip((psi, chi), A0)]
    h1 = [febe(1, s, a) for s, a in zip((psi, chi), A0)]
    Ah = A(*h1)
    h2 = [febe(1, s, a) for s, a in zip(h1, Ah)]
    s = [2.0 * h - f for h, f in zip(h2, full)]
    prev = A0
    for _ in range(n - 1):
        now = A(*s)
        nxt = []
        for x, an, ap in zip(s, now, prev):
            o = plan.empty_spec()
            plan.step_abcn(x, an, ap, o)
            nxt.append(o)
        s, prev = nxt, now
    return s, prev


@pytest.mark.parametrize("with_closure", [False, True])
def test_tp_advance_matches_single_steps(with_closure):
    m = _gpu()
    _say("tp_advance vs single steps, closure", with_closure)
    nr, nphi, nz = 16, 8, 8
    g = Grid(nr, nphi, nz, 1.0)
    plan = m.Plan(nr, nphi, nz, 1.0)
    plan.step_setup(0.01, 1e-6, 8, 1e-3)
    cl = None
    if with_closure:
        cl = m.Closure(plan, max_batch=64, beta=1e30)
        params = synth.closure_init(5) * 0.5
        cl.set_params(params)
        cl.set_scales(np.full(258, 10.0, np.float32), np.full(256, 1e-4, np.float32))
    sp, sc = _state(g, 80)
    U = (0.0, 1.0, 0.0)
    ref_s, ref_prev = _manual(plan, _dev(sp), _dev(sc), 4, U, cl)
    psi, chi = _dev(sp), _dev(sc)
    hp, hc = plan.empty_spec(), plan.empty_spec()
    plan.advance(psi, chi, hp, hc, 4, start=1, U=U, closure=cl)
    torch.cuda.synchronize()
    assert torch.equal(psi, ref_s[0]) and torch.equal(chi, ref_s[1])
    assert torch.equal(hp, ref_prev[0]) and torch.equal(hc, ref_prev[1])
    # split calls continue from the history
    psi2, chi2 = _dev(sp), _dev(sc)
    plan.advance(psi2, chi2, hp, hc, 1, start=1, U=U, closure=cl)
    plan.advance(psi2, chi2, hp, hc, 3, start=0, U=U, closure=cl)
    torch.cuda.synchronize()
    assert torch.equal(psi2, psi) and torch.equal(chi2, chi)
    if cl is not None:
        calls, fbs = cl.stats()
        assert fbs == 0 and calls > 0
