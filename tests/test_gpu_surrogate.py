"""Parity of the pre-filter kernels (through the C ABI) with the FP64 NumPy oracle."""
import numpy as np
import pytest
import torch

from oracle import surrogate as S
from paper_2304_09953_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09953_amd import pipeline as P
    from paper_2304_09953_amd import surrogate as SG
    return P, SG


def _bits_to_f64(t: torch.Tensor) -> np.ndarray:
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-30))


def _check_counts(got_log1p, ligs, status=None):
    """GPU features (log1p of counts, unscaled) against the FP64 oracle: type counts and rotatable
    counts exactly; each histogram row exactly except for pairs the oracle flags as lying within
    1e-5 A of a bin edge (each may sit in either neighbouring bin)."""
    ref, near = S.raw_features_flagged(ligs, status)
    cnt = np.round(np.expm1(got_log1p.astype(np.float64))).reshape(-1, 16, 32)
    assert np.allclose(np.expm1(got_log1p.astype(np.float64)).reshape(-1, 16, 32), cnt, atol=1e-2)
    ref = ref.reshape(-1, 16, 32)
    assert np.array_equal(cnt[:, :, 0], ref[:, :, 0])
    assert np.array_equal(cnt[:, :, 31], ref[:, :, 31])
    diff = np.abs(cnt[:, :, 1:31] - ref[:, :, 1:31]).sum(axis=2)
    assert np.all(diff <= 2 * near), np.argwhere(diff > 2 * near)[:5]
    assert np.array_equal(cnt[:, :, 1:31].sum(axis=2), ref[:, :, 1:31].sum(axis=2))  # moves stay in the row
    say(f"features: {int(near.sum())} flagged pairs, {int((diff > 0).sum())} rows differ by them")
    same = (diff == 0).reshape(-1)
    return ref.reshape(-1, 512), same


def test_features_match_oracle(env):
    P, SG = env
    ligs = I.make_ligands(300, I.DIST_HEAVY_TAIL, 16, stream="test")
    say("features of 300 ligands (n up to 120)")
    lib = P.DeviceLibrary(ligs)
    F, Fb = SG.features(lib)
    got = F.cpu().numpy()
    ref_raw, same_row = _check_counts(got, ligs)
    ref = np.log1p(ref_raw)
    # rows with the same counts: log1p in FP32 against FP64
    g64 = got.astype(np.float64).reshape(-1, 16, 32)[same_row.reshape(-1, 16)]
    assert np.allclose(g64, ref.reshape(-1, 16, 32)[same_row.reshape(-1, 16)], rtol=2e-7, atol=1e-7)
    assert np.array_equal(_bits_to_f64(Fb), S.bf16_round(got))
    mean, istd = SG.feature_stats(F)
    m_ref, i_ref = S.feature_stats(ref)
    assert np.allclose(mean.cpu().numpy(), m_ref, rtol=1e-5, atol=1e-5)
    assert np.allclose(istd.cpu().numpy(), i_ref, rtol=1e-4, atol=1e-5)
    Fn, _ = SG.features(lib, mean, istd)
    assert np.allclose(Fn.cpu().numpy(), S.normalise(got.astype(np.float64), mean.cpu().numpy().astype(np.float64),
                                                     istd.cpu().numpy().astype(np.float64)), rtol=1e-4, atol=1e-4)


@pytest.mark.timeout(300)
def test_features_at_library_scale(env):
    """The first 20000 ligands of the 100k-ligand benchmark library (the pre-filter's inputs at their
    real distribution, 15-70 atoms): every count against the oracle."""
    P, SG = env
    ligs = I.workload("pocket96-lib100k").ligands(n_lig=20000)
    say("features of the benchmark library's first 20000 ligands")
    F, _ = SG.features(P.DeviceLibrary(ligs), bf16=False)
    _check_counts(F.cpu().numpy(), ligs)


def test_invalid_ligands_get_zero_features(env):
    P, SG = env
    from test_gpu_parity import _edge_library
    ligs = _edge_library()
    lib = P.DeviceLibrary(ligs)
    st = lib.status.cpu().numpy()
    F, _ = SG.features(lib)
    F = F.cpu().numpy()
    assert np.all(F[st != 0] == 0)
    ok = np.flatnonzero((st == 0) & (np.array([t.max() for t in (ligs.ligand(i)[1] for i in range(ligs.n_lig))]) < 16))
    _check_counts(F[ok], ligs.subset(ok))


def test_features_of_a_32_type_pack(env):
    """A library packed with 32 types: ligands holding a type >= 16 have no feature row for it and
    get zero features (nothing is written past the 16-row histogram); the rest match the oracle."""
    P, SG = env
    a = I.make_ligands(32, I.DIST_DRUGLIKE, 16, stream="test")
    b = I.make_ligands(32, I.DIST_DRUGLIKE, 32, stream="test")
    ligs = I.from_parts([x.ligand(i) for i in range(32) for x in (a, b)], 32)
    say("features of a 32-type pack, 64 ligands")
    lib = P.DeviceLibrary(ligs)
    assert np.all(lib.status.cpu().numpy() == 0)
    tmax = np.array([ligs.ligand(i)[1].max() for i in range(ligs.n_lig)])
    assert (tmax >= 16).any() and (tmax < 16).any()
    F = SG.features(lib, n_types=16)[0].cpu().numpy()
    assert np.all(F[tmax >= 16] == 0)
    _check_counts(F, ligs)


@pytest.mark.parametrize("dims,batch", [((64, 64, 64), 40), ((512, 1024, 1024), 1024), ((128, 192, 64), 97),
                                        ((512, 1024, 1024), 5000)])
def test_forward_matches_bf16_mirror(env, dims, batch):
    P, SG = env
    d, h1, h2 = dims
    rng = np.random.default_rng(d + batch)
    init = I.mlp_init(d, h1, h2, seed=d)
    init[d * h1:d * h1 + h1] = rng.normal(size=h1) * 0.1  # non-zero biases
    m = SG.Model(init, d, h1, h2)
    X = rng.normal(size=(batch, d)).astype(np.float32)
    xb = torch.as_tensor(S.bf16_bits(X).view(np.int16)).cuda()
    say(f"forward {dims} batch {batch}")
    y = m.forward(xb).cpu().numpy()
    y_ref, _ = S.forward(S.Params(d, h1, h2), init.astype(np.float64), X)
    say(f"forward rel err {_rel(y, y_ref):.3g}")
    assert _rel(y, y_ref) < 2e-3


@pytest.mark.parametrize("dims", [(512, 1024, 1024), (128, 256, 128)])
def test_large_batches_equal_small_ones(env, dims):
    # every row's output depends on that row alone and takes the same MFMA sequence over K whatever
    # the batch, so a large batch and its chunks agree bit for bit
    P, SG = env
    d, h1, h2 = dims
    rng = np.random.default_rng(11)
    init = I.mlp_init(d, h1, h2, seed=3)
    init[d * h1:d * h1 + h1] = rng.normal(size=h1) * 0.1
    m = SG.Model(init, d, h1, h2)
    n = 9000  # 35 row blocks of 256 and a ragged tail
    xb = torch.as_tensor(S.bf16_bits(rng.normal(size=(n, d)).astype(np.float32)).view(np.int16)).cuda()
    say(f"forward {dims}: batch {n} against chunks of 1500")
    big = m.forward(xb)
    small = torch.cat([m.forward(xb[s:s + 1500]) for s in range(0, n, 1500)])
    assert torch.equal(big, small)


def test_backward_and_adam_match_oracle(env):
    P, SG = env
    d, h1, h2, B = 512, 1024, 1024, 256
    rng = np.random.default_rng(5)
    init = I.mlp_init(d, h1, h2, seed=7)
    init[d * h1:d * h1 + h1] = rng.normal(size=h1) * 0.05
    m = SG.Model(init, d, h1, h2)
    X = rng.normal(size=(B, d)).astype(np.float32)
    t = rng.normal(size=B).astype(np.float32)
    xb = torch.as_tensor(S.bf16_bits(X).view(np.int16)).cuda()
    tt = torch.as_tensor(t).cuda()
    loss = torch.empty(1, device="cuda")
    say("backward 512-1024-1024 batch 256")
    m.backward(xb, tt, loss)
    g = m.grad.cpu().numpy().astype(np.float64)
    Pm = S.Params(d, h1, h2)
    l_ref, g_ref = S.backward(Pm, init.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    assert abs(loss.item() - l_ref) <= 1e-3 * max(1.0, l_ref)
    for name, gp, gr in zip(Pm.shapes, Pm.split(g).values(), Pm.split(g_ref).values()):
        say(f"grad {name[0]} rel err {_rel(gp, gr):.3g}")
        assert _rel(gp, gr) < 5e-3, name
    say("Adam step")
    m.adam(1e-3)
    w1 = m.master.cpu().numpy().astype(np.float64)
    w_ref, _, _ = S.adam(init.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1)
    assert np.allclose(w1, w_ref, rtol=1e-6, atol=1e-9)
    assert np.array_equal(_bits_to_f64(m.bf16[:d * h1]), S.bf16_round(w1[:d * h1]))


def test_training_overfits_a_small_set(env):
    P, SG = env
    rng = np.random.default_rng(3)
    n, d = 512, 512
    X = rng.normal(size=(n, d)).astype(np.float32)
    t = (np.tanh(X[:, :8].sum(1) / 3) + 0.1 * rng.normal(size=n)).astype(np.float32)
    m = SG.Model(I.mlp_init(d, 1024, 1024, seed=1))
    xb = torch.as_tensor(S.bf16_bits(X).view(np.int16)).cuda()
    say("train 512 samples x 40 epochs")
    hist = SG.train(m, xb, torch.as_tensor(t).cuda(), epochs=40, batch=128, lr=1e-3, seed=0)
    say(f"loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    assert hist[-1] < 0.1 * hist[0]
    y = m.predict(xb).cpu().numpy()
    assert S.r2(y, t) > 0.9


def test_ensemble_average_on_the_device(env):
    P, SG = env
    rng = np.random.default_rng(8)
    for m, n in ((1, 5), (4, 70001), (7, 1000)):
        say(f"surr_average of {m} members x {n}")
        y = rng.normal(size=(m, n)).astype(np.float32)
        got = SG.average(torch.as_tensor(y).cuda()).cpu().numpy()
        ref = y.astype(np.float64).mean(0)
        assert np.allclose(got, ref, rtol=1e-6, atol=1e-6)
        s = np.zeros(n, np.float32)
        for k in range(m):  # the stated order: FP32 sums over members in order, then one division
            s = (s + y[k]).astype(np.float32)
        assert np.array_equal(got, (s / np.float32(m)).astype(np.float32))
