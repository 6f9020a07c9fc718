"""GPU parity of the learned picker's kernels against the float64 reference
(oracle/mlp_ref.py): sketch, forward, gradient, Adam, training determinism and
the masked argmin pick.  Exact bin counts.

Tolerance of the FP32 kernels against float64.  The reference runs on the
same fp32-rounded parameters and inputs the kernels receive, so the only
difference is FP32 rounding inside the kernels.  Every output or gradient
element is a composition of sums; to first order in the unit roundoff
u = 2^-24, rounding changes element e by at most K u A_e, where A_e is the
same element computed with every factor replaced by its absolute value (and
ReLU masks kept) and K is the total length of the sums on its dependency
chain (forward 34 + 64 + 64, backward 62 + 64, the batch sum B).  The test
allows |got - want| <= 1e-4 |want| + 2 K u A_e: relative tolerance 1e-4 where
no cancellation occurs, and the derived bound (with a factor 2 of slack) where
it does."""
import sys

import numpy as np
import pytest

from oracle import mlp_ref as M
from paper_2609_00843_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
SIZES = (34, 64, 64, 62)
NPARAM = sum(SIZES[i + 1] * SIZES[i] + SIZES[i + 1] for i in range(3))   # 10430


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def r():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_00843_amd import rtcdf
    return rtcdf


def _init(seed):
    rng = np.random.default_rng(seed)
    p = {}
    for i in range(3):
        p[f"W{i + 1}"] = rng.normal(0, np.sqrt(2.0 / SIZES[i]), size=(SIZES[i + 1], SIZES[i]))
        p[f"b{i + 1}"] = rng.normal(0, 0.05, size=SIZES[i + 1])
    return p


def _flat(p):
    return np.concatenate([p[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def _unflat(v):
    out, o = {}, 0
    for i in range(3):
        for k, shape in ((f"W{i + 1}", (SIZES[i + 1], SIZES[i])), (f"b{i + 1}", (SIZES[i + 1],))):
            sz = int(np.prod(shape))
            out[k] = v[o:o + sz].reshape(shape)
            o += sz
    return out


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _batch(seed, B):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, 34))
    T = rng.normal(size=(B, SIZES[3]))
    Mk = np.ones((B, SIZES[3]))
    Mk[:, [38, 41, 44, 46, 47, 49, 50, 52, 53]] = 0.0      # the invalid grid points
    Mk[rng.random(size=(B, SIZES[3])) < 0.05] = 0.0
    return X, T, Mk


@pytest.mark.parametrize("dist,n,R", [("uniform", 10 ** 6, 128), ("normal", 3_000_001, 70000),
                                      ("all_equal", 5000, 1 << 18), ("zipf", 777, 1000),
                                      ("uniform", 4096, 33), ("normal", 12345, 1 << 28)])
def test_sketch(r, dist, n, R):
    lo = -12345
    A = inputs.make(dist, n, lo, lo + R, 11)
    _say(f"sketch {dist} n={n} R={R}")
    got = r.sketch(torch.from_numpy(A).cuda(), lo, lo + R).cpu().numpy().astype(np.float64)
    want = M.sketch(A, lo, lo + R, samples=4096, bins=32)
    assert np.allclose(got[:2], want[:2], rtol=1e-6, atol=0)
    S = min(4096, n)
    assert np.array_equal(np.rint(got[2:] * S), np.rint(want[2:] * S))   # identical bin counts



@pytest.mark.parametrize("k", range(30))
def test_sketch_random(r, k):
    """The sketch of random arrays (n from 1 to 3 x 10^6, R from 1 to 2^28,
    minVal down to INT32_MIN and ranges up to 2^31): the same features as
    the float64 reference and identical bin counts."""
    rng = np.random.default_rng(inputs.case_seed(108, k))
    n = int(round(10 ** rng.uniform(0, 6.5)))
    R = max(1, int(round(2 ** rng.uniform(0, 28))))
    u = rng.random()
    lo = -(1 << 31) if u < 0.2 else ((1 << 31) - R if u < 0.4 else int(rng.integers(-(1 << 31), (1 << 31) - R + 1)))
    dist = str(rng.choice(["uniform", "normal", "all_equal", "zipf"]))
    A = inputs.make(dist, n, lo, lo + R, inputs.case_seed(109, k))
    _say(f"sketch random {k}: {dist} n={n} [{lo},{lo + R})")
    got = r.sketch(torch.from_numpy(A).cuda(), lo, lo + R).cpu().numpy().astype(np.float64)
    want = M.sketch(A, lo, lo + R, samples=4096, bins=32)
    assert np.allclose(got[:2], want[:2], rtol=1e-6, atol=0)
    S = min(4096, n)
    assert np.array_equal(np.rint(got[2:] * S), np.rint(want[2:] * S))


U32 = 2.0 ** -24


def _f32(a):
    """The float64 value of a's float32 rounding (what the kernels receive)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _magnitudes(p, X, T, Mk):
    """Absolute-value forms of the forward output and of every gradient
    element (ReLU masks of the true forward pass kept): the A_e of the
    module docstring."""
    A = {k: np.abs(v) for k, v in p.items()}
    Y, (_, Z1, _, Z2, _) = M.forward(p, X)
    H1a = (np.abs(X) @ A["W1"].T + A["b1"]) * (Z1 > 0)
    H2a = (H1a @ A["W2"].T + A["b2"]) * (Z2 > 0)
    Ya = H2a @ A["W3"].T + A["b3"]
    dYa = 2.0 * Mk * (np.abs(Y - T) + Ya) / Mk.sum()
    g = {"W3": dYa.T @ H2a, "b3": dYa.sum(axis=0)}
    dZ2a = (dYa @ A["W3"]) * (Z2 > 0)
    g["W2"], g["b2"] = dZ2a.T @ H1a, dZ2a.sum(axis=0)
    dZ1a = (dZ2a @ A["W2"]) * (Z1 > 0)
    g["W1"], g["b1"] = dZ1a.T @ np.abs(X), dZ1a.sum(axis=0)
    return Ya, _flat(g)


@pytest.mark.parametrize("B", [1, 2, 63, 64, 65, 300, 1000, 2500])
def test_forward_and_gradient(r, B):
    """Forward output, gradient and loss against the float64 reference within
    the bound above, from one sample to more than the training sets hold (the
    forward and delta kernels take one sample per workgroup; the weight
    gradient sums every sample per parameter, so its rounding grows with B)."""
    p = {k: _f32(v) for k, v in _init(1).items()}
    X, T, Mk = (_f32(a) for a in _batch(2, B))
    P = _dev(_flat(p))
    _say("forward")
    Y = r.mlp_forward(P, _dev(X)).cpu().numpy()
    Yr, cache = M.forward(p, X)
    Ya, Ga = _magnitudes(p, X, T, Mk)
    k_fwd = 34 + 64 + 64
    assert np.all(np.abs(Y - Yr) <= 1e-4 * np.abs(Yr) + 2 * k_fwd * U32 * Ya)
    _say("gradient")
    G, L = r.mlp_gradient(P, _dev(X), _dev(T), _dev(Mk))
    gr = _flat(M.backward(p, cache, Yr, T, Mk))
    g = G.cpu().numpy().astype(np.float64)
    k_bwd = k_fwd + SIZES[3] + 64 + B
    bound = 1e-4 * np.abs(gr) + 2 * k_bwd * U32 * Ga
    worst = int(np.argmax(np.abs(g - gr) - bound))
    assert np.all(np.abs(g - gr) <= bound), (worst, g[worst], gr[worst], bound[worst])
    # Batch sums of 300 terms of both signs cancel (A_e is ~10^3 |g_e| at the
    # median), which is what the K u A_e term covers; the stated relative
    # tolerance alone holds for all but a few elements (a CPU emulation of
    # sequential FP32 sums gives 99.9 %).
    assert np.mean(np.abs(g - gr) <= 1e-4 * np.abs(gr)) >= 0.99
    assert float(L.cpu()[0]) == pytest.approx(M.loss(Yr, T, Mk), rel=1e-4)


def test_adam_step(r):
    rng = np.random.default_rng(3)
    p = {"w": rng.normal(size=NPARAM)}
    g = {"w": rng.normal(size=NPARAM)}
    m = {"w": rng.normal(size=NPARAM) * 0.1}
    v = {"w": np.abs(rng.normal(size=NPARAM)) * 0.01}
    P, Gd, Md, Vd = _dev(p["w"]), _dev(g["w"]), _dev(m["w"]), _dev(v["w"])
    _say("adam")
    r.mlp_adam_step(P, Gd, Md, Vd, 7, lr=1e-2)
    # the kernel receives float hyperparameters: give the reference the same values
    f32 = lambda x: float(np.float32(x))
    M.adam_step(p, g, m, v, 7, lr=f32(1e-2), beta1=f32(0.9), beta2=f32(0.999), eps=f32(1e-8))
    assert np.allclose(P.cpu().numpy(), p["w"], rtol=1e-5, atol=1e-6)
    assert np.allclose(Md.cpu().numpy(), m["w"], rtol=1e-5, atol=1e-7)
    assert np.allclose(Vd.cpu().numpy(), v["w"], rtol=1e-5, atol=1e-9)


def test_training_is_deterministic_and_learns(r):
    p0 = _flat(_init(4))
    X, T, Mk = _batch(5, 500)
    Xd, Td, Md = _dev(X), _dev(T * 0.1 + X[:, :1] * 0.5), _dev(Mk)
    finals = []
    for rep in range(2):
        P = _dev(p0)
        m = torch.zeros_like(P)
        v = torch.zeros_like(P)
        hist = torch.empty(200, dtype=torch.float32, device="cuda")
        _say(f"train run {rep}")
        r.mlp_train(P, m, v, 0, Xd, Td, Md, 200, 3e-3, loss_history=hist)
        torch.cuda.synchronize()
        h = hist.cpu().numpy()
        assert h[-1] < 0.5 * h[0]
        finals.append(P.cpu().numpy())
    assert np.array_equal(finals[0], finals[1])


def test_pick(r):
    p = _init(6)
    rng = np.random.default_rng(7)
    norm = np.concatenate([rng.normal(size=34) * 0.1, 0.5 + rng.random(size=34)])
    _, valid = r.config_grid()
    validd = torch.tensor(np.array(valid, dtype=np.uint8), device="cuda")
    for dist, n, R in (("uniform", 100_000, 4096), ("normal", 50_000, 300), ("zipf", 9999, 65536)):
        A = inputs.make(dist, n, 0, R, 8)
        _say(f"pick {dist}")
        idx, pred = r.mlp_pick(torch.from_numpy(A).cuda(), 0, R, _dev(_flat(p)), _dev(norm), validd)
        pred = pred.cpu().numpy()
        f = (M.sketch(A, 0, R) - norm[:34]) / norm[34:]
        want, _ = M.forward(p, f[None, :])
        assert np.allclose(pred, want[0], rtol=1e-4, atol=1e-4 * np.abs(want).max())
        # the argmin is taken in the kernel's precision: compare on its own outputs
        assert int(idx.cpu()[0]) == M.pick(pred, valid)


@pytest.mark.parametrize("margin", [0.0, 0.02, 1e30])
def test_learned_pick_applies_margin(r, tmp_path, margin):
    """LEARNED mode keeps the static configuration unless the network predicts
    at least the model's margin of gain: the library's choice (its grid
    index) equals learn.decide applied to the pick kernel's own predictions."""
    from paper_2609_00843_amd import learn, tune
    p = _flat(_init(8))
    rng = np.random.default_rng(9)
    mu, sd = rng.normal(size=34) * 0.1, 0.5 + rng.random(size=34)
    path = str(tmp_path / "m.bin")
    learn.save_model(path, p, mu, sd, (10.0, 30.0, 4.0, 20.0), margin=margin, zmax=0.0)
    pts, valid = tune.grid()
    r.load_model(path)
    old = r.get_config_mode()
    try:
        for dist, n, R in (("uniform", 2_000_000, 4096), ("normal", 1_500_000, 70000), ("zipf", 3_000_000, 300)):
            A = inputs.make(dist, n, 0, R, 10)
            d = torch.from_numpy(A).cuda()
            _say(f"learned pick {dist} margin={margin}")
            r.set_config_mode(r.CONFIG_DEFAULT)
            r.pick_config(n, 0, R)
            static = r.last_pick()[0]
            r.set_config_mode(r.CONFIG_LEARNED)
            r.clear_pick_cache()
            cfg = r.pick_config(n, 0, R, keys_in=d)
            got, source = r.last_pick()
            norm = np.concatenate([mu, sd])
            validd = torch.tensor(np.array(valid, dtype=np.uint8), device="cuda")
            _, pred = r.mlp_pick(d, 0, R, _dev(p), _dev(norm), validd)
            # the library compares in FP32: so does the reference here
            want = learn.decide(pred.cpu().numpy(), np.array(valid), static, np.float32(margin))
            assert got == want
            assert source in (r.PICK_NETWORK, r.PICK_NETWORK_KEPT_STATIC)
            if want >= tune.PLAIN_POINTS:   # an option point: static knobs with its flags
                assert cfg.flags == pts[want][3] and cfg.tile_width > 0
            if margin >= 1e30:
                assert got == static and source == r.PICK_NETWORK_KEPT_STATIC
            # the same buffer again: the decision is reused without a pick
            r.pick_config(n, 0, R, keys_in=d)
            assert r.last_pick() == (got, r.PICK_CACHED)
    finally:
        r.set_config_mode(old)
        r.unload_model()


def test_learned_pick_feature_gate(r, tmp_path):
    """A sketch farther than zmax from the training mean is not judged by the
    network: with the exhaustive fallback off the static configuration is
    kept whatever the network prefers; within zmax the network decides."""
    from paper_2609_00843_amd import learn, tune
    p = _flat(_init(8))
    pts, valid = tune.grid()
    A = inputs.make("zipf", 2_000_000, 0, 50000, 12)
    d = torch.from_numpy(A).cuda()
    feats = M.sketch(A, 0, 50000)
    mu, sd = np.zeros(34), np.ones(34)
    z = float(np.abs(feats - mu).max())          # the array's distance in sd units
    old = r.get_config_mode()
    try:
        r.set_learned_fallback(False)
        r.set_config_mode(r.CONFIG_DEFAULT)
        r.pick_config(A.size, 0, 50000)
        static = r.last_pick()[0]
        _, pred = r.mlp_pick(d, 0, 50000, _dev(p), _dev(np.concatenate([mu, sd])),
                             torch.tensor(np.array(valid, dtype=np.uint8), device="cuda"))
        free = learn.decide(pred.cpu().numpy(), np.array(valid), static, np.float32(0.0))
        for zmax, want in ((z * 0.5, static), (z * 2.0, free)):
            path = str(tmp_path / f"m{zmax}.bin")
            learn.save_model(path, p, mu, sd, (10.0, 30.0, 4.0, 20.0), margin=0.0, zmax=zmax)
            r.load_model(path)
            r.set_config_mode(r.CONFIG_LEARNED)
            _say(f"feature gate zmax={zmax:.3f} (array at {z:.3f})")
            r.pick_config(A.size, 0, 50000, keys_in=d)
            assert r.last_pick()[0] == want
            r.unload_model()
    finally:
        r.set_learned_fallback(True)
        r.set_config_mode(old)


def test_learned_fallback_autotunes_untrusted_arrays(r, tmp_path):
    """Where the network is not trusted the grid is timed exhaustively: the
    decision's source is AUTOTUNED, its index a valid grid point, the sort
    with it equals the oracle's, and a second array of the same shape class
    reuses the result (no second timing: much faster than the first)."""
    import time
    from paper_2609_00843_amd import learn, tune
    import oracle
    p = _flat(_init(8))
    pts, valid = tune.grid()
    mu, sd = np.zeros(34), np.ones(34)
    path = str(tmp_path / "m.bin")
    learn.save_model(path, p, mu, sd, (10.0, 30.0, 4.0, 20.0), margin=0.0, zmax=1e-3)   # nothing trusted
    r.load_model(path)
    old = r.get_config_mode()
    try:
        r.set_config_mode(r.CONFIG_LEARNED)
        r.clear_pick_cache()
        walls = []
        for seed in (20, 21):
            A = inputs.make("zipf", 1_000_000, 0, 20000, seed)
            d = torch.from_numpy(A).cuda()
            _say(f"fallback pick seed={seed}")
            t0 = time.perf_counter()
            r.pick_config(A.size, 0, 20000, keys_in=d)
            walls.append(time.perf_counter() - t0)
            idx, source = r.last_pick()
            assert source == r.PICK_AUTOTUNED and valid[idx]
            out = r.sort(d, 0, 20000)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), oracle.sort(A, 0, 20000))
        assert walls[1] < 0.5 * walls[0]
    finally:
        r.set_config_mode(old)
        r.unload_model()
        r.clear_pick_cache()
