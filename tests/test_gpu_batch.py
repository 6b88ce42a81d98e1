"""Batched solves (mag_weighting_batch, mag_tplus_batch): every item against the
single-call result and the CPU oracle, on clouds of uneven n."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def test_weighting_batch_uneven(mag):
    clouds = [W.gaussian_mixture(n, 3, seed=s) for s, n in enumerate([300, 1000, 777, 256, 1, 2, 1500])]
    X, offs = W.pack_clouds(clouds)
    ts = [30.0, 12.0, 45.0, 5.0, 2.0, 1.0, 25.0]
    w, Ms, infos = mag.weighting_batch(dev(X), offs, ts)
    w = w.cpu().numpy()
    for b, (Xb, t) in enumerate(zip(clouds, ts)):
        wb = w[offs[b]:offs[b + 1]]
        assert infos[b]["status"] == 0
        assert np.abs(oracle.residual(Xb, t, wb)).max() <= 1e-12, b
        ref = oracle.weighting(Xb, t)
        assert abs(Ms[b] - ref.M) / abs(ref.M) <= 1e-10
        # the single solve takes other correction steps (plain refinement first),
        # so the two agree to the solves' accuracy, not bitwise
        single = mag.weighting(dev(Xb), t)
        ws = single.w.cpu().numpy()
        assert np.abs(wb - ws).max() <= 1e-10 * max(1.0, np.abs(ws).max())
        assert infos[b]["argmin_w"] == int(np.argmin(wb))


@pytest.mark.parametrize("m", [2, 7, 16, 17, 30])
def test_weighting_batch_tile_edges(mag, m):
    # clouds on and around the 128/256 tile edges in one batch, several dimensions
    # (the batched products' generic paths above 16)
    sizes = [127, 128, 129, 255, 256, 257, 511, 513, 3]
    clouds = [W.gaussian(n, m, seed=60 + i) for i, n in enumerate(sizes)]
    X, offs = W.pack_clouds(clouds)
    ts = [float(W.gaussian_cutoff_estimate(n, m)) * f for n, f in zip(sizes, [0.3, 1, 3, 0.5, 2, 1, 0.7, 1.5, 1])]
    w, Ms, infos = mag.weighting_batch(dev(X), offs, ts)
    w = w.cpu().numpy()
    for b, (Xb, t) in enumerate(zip(clouds, ts)):
        wb = w[offs[b]:offs[b + 1]]
        assert infos[b]["status"] == 0, b
        assert np.abs(oracle.residual(Xb, t, wb)).max() <= 1e-12, (m, b)
        ref = oracle.weighting(Xb, t)
        assert abs(Ms[b] - ref.M) / abs(ref.M) <= 1e-10, (m, b)


def test_weighting_batch_t_sweep_shared_rows(mag):
    # several scales of one cloud: items may share rows of X
    Xc = W.gaussian(900, 3, seed=2)
    ts = [0.5, 1.0, 2.0, 4.0, 8.0]
    X = np.concatenate([Xc] * len(ts))
    offs = np.arange(len(ts) + 1) * 900
    w, Ms, infos = mag.weighting_batch(dev(X), offs, ts)
    w = w.cpu().numpy()
    for b, t in enumerate(ts):
        ref = oracle.weighting(Xc, t)
        assert abs(Ms[b] - ref.M) / abs(ref.M) <= 1e-10
        assert np.abs(oracle.residual(Xc, t, w[900 * b:900 * (b + 1)])).max() <= 1e-12


def test_weighting_batch_repeat_deterministic(mag):
    clouds = [W.gaussian(n, 3, seed=n) for n in (400, 640)]
    X, offs = W.pack_clouds(clouds)
    a = mag.weighting_batch(dev(X), offs, [3.0, 3.0])[0].cpu().numpy()
    b = mag.weighting_batch(dev(X), offs, [3.0, 3.0])[0].cpu().numpy()
    assert np.array_equal(a, b)


def test_tplus_batch_vs_single_and_oracle(mag):
    clouds = W.mixture_clouds(B=6, m=3, seed=11, n_lo=300, n_hi=900)
    clouds.append(W.centre_kgon(8, m=3))
    X, offs = W.pack_clouds(clouds)
    tps, w, infos = mag.tplus_batch(dev(X), offs, want_w=True)
    w = w.cpu().numpy()
    for b, Xb in enumerate(clouds):
        single = mag.tplus(dev(Xb))
        assert infos[b]["no_sign_change"] == 0
        assert abs(tps[b] - single.t_plus) / single.t_plus <= 2.5e-6
        wb = w[offs[b]:offs[b + 1]]
        assert wb.min() >= 0
        assert np.abs(oracle.residual(Xb, tps[b], wb)).max() <= 1e-12
        if b < 3:
            ref = oracle.tplus(Xb)
            assert abs(tps[b] - ref.t_plus) / ref.t_plus <= 2.5e-6
        print(b, len(Xb), tps[b], infos[b]["solves"], infos[b]["newton_steps"])


def test_tplus_batch_ridders_vs_single(mag):
    clouds = W.mixture_clouds(B=5, m=3, seed=12, n_lo=300, n_hi=800)
    clouds.append(W.centre_kgon(12, m=3))
    X, offs = W.pack_clouds(clouds)
    tps, w, infos = mag.tplus_batch(dev(X), offs, want_w=True, method="ridders")
    w = w.cpu().numpy()
    for b, Xb in enumerate(clouds):
        single = mag.tplus(dev(Xb), method="ridders")
        assert infos[b]["no_sign_change"] == 0
        # the same rules, one evaluation per batched solve (the batched products sum in
        # another order, so a decision next to the root can differ)
        assert abs(tps[b] - single.t_plus) / single.t_plus <= 2.5e-6
        wb = w[offs[b]:offs[b + 1]]
        assert wb.min() >= 0
        assert np.abs(oracle.residual(Xb, tps[b], wb)).max() <= 1e-12
        print(b, len(Xb), tps[b], single.t_plus, infos[b]["solves"], single.info["solves"])


def test_tplus_batch_no_sign_change_items(mag):
    rng = np.random.default_rng(4)
    s_pos = np.linspace(0.0, 1.0, 200) + rng.random(200) * (0.1 / 200)
    line = np.ascontiguousarray(s_pos[:, None] * np.array([0.6, 0.8, 0.0])[None, :])
    clouds = [line, np.zeros((1, 3)), W.gaussian_mixture(400, 3, seed=5)]
    X, offs = W.pack_clouds(clouds)
    tps, _, infos = mag.tplus_batch(dev(X), offs, max_extend=0)
    assert infos[0]["no_sign_change"] == 1 and tps[0] == 0.0
    assert infos[1]["no_sign_change"] == 1 and tps[1] == 0.0
    assert infos[2]["no_sign_change"] == 0 and tps[2] > 0


# ---- the batched cutoff workload at full scale: 64 mixture clouds, n ~ U{1000..6000}

@pytest.fixture(scope="module")
def mixture64(mag):
    clouds = W.mixture_clouds(B=64, m=3, seed=0)
    X, offs = W.pack_clouds(clouds)
    tps, w, infos = mag.tplus_batch(dev(X), offs, want_w=True)
    return clouds, offs, tps, w.cpu().numpy(), infos


def test_tplus_batch_mixture64_signs(mag, mixture64):
    # every cloud's cutoff: w >= 0 at t_+(1 + 1e-5) and min w < 0 at t_+(1 - 1e-5),
    # each decided by the FP64 dense comparator (FP64 Z + rocSOLVER Cholesky), a
    # solver the search does not use; and w(t_+) returned by the search solves
    # Z w = 1 (oracle Dot2 residual on sampled rows)
    clouds, offs, tps, w, infos = mixture64
    assert len(clouds) == 64
    sizes = [len(c) for c in clouds]
    assert min(sizes) >= 1000 and max(sizes) <= 6000
    for b, Xb in enumerate(clouds):
        assert infos[b]["no_sign_change"] == 0, b
        tp = tps[b]
        assert 0 < tp <= infos[b]["t_bound"]
        Xd = dev(Xb)
        above = mag.weighting(Xd, tp * (1 + 1e-5), solver="fp64_dense").info["min_w"]
        below = mag.weighting(Xd, tp * (1 - 1e-5), solver="fp64_dense").info["min_w"]
        assert above >= 0 and below < 0, (b, len(Xb), tp, above, below)
        wb = w[offs[b]:offs[b + 1]]
        assert wb.min() >= 0
        rows = np.random.default_rng(b).choice(len(Xb), size=32, replace=False)
        assert np.abs(oracle.residual(Xb, tp, wb, rows)).max() <= 1e-12
    print("mixture64: n in [%d, %d], t_+ in [%.4f, %.4f], solves %d" %
          (min(sizes), max(sizes), min(tps), max(tps), sum(i["solves"] for i in infos)))


@pytest.mark.parametrize("rank", [0, 1, 2])
def test_tplus_batch_mixture64_vs_oracle(mag, mixture64, rank):
    # the three smallest clouds against the oracle's bisection and the single call
    clouds, offs, tps, w, infos = mixture64
    b = int(np.argsort([len(c) for c in clouds])[rank])
    Xb = clouds[b]
    ref = oracle.tplus(Xb)
    single = mag.tplus(dev(Xb))
    print(f"cloud {b} n={len(Xb)}: batch {tps[b]:.9g} single {single.t_plus:.9g} oracle {ref.t_plus:.9g}")
    assert abs(tps[b] - ref.t_plus) / ref.t_plus <= 2.5e-6
    assert abs(single.t_plus - ref.t_plus) / ref.t_plus <= 2.5e-6
    assert abs(infos[b]["t_bound"] - ref.t_bound) <= 1e-12 * ref.t_bound


# ---- panel grouping of the batched factorisation and its autotuner

def test_batch_groupings_against_oracle(mag):
    clouds = [W.gaussian_mixture(n, 3, seed=40 + i) for i, n in enumerate([700, 1300, 2600, 257])]
    X, offs = W.pack_clouds(clouds)
    ts = [20.0, 35.0, 50.0, 8.0]
    res = {}
    try:
        for group in (1, 2):
            mag.tune_batch_group(max(len(c) for c in clouds), group)
            w, Ms, infos = mag.weighting_batch(dev(X), offs, ts)
            w = w.cpu().numpy()
            for b, (Xb, t) in enumerate(zip(clouds, ts)):
                wb = w[offs[b]:offs[b + 1]]
                assert infos[b]["status"] == 0
                assert np.abs(oracle.residual(Xb, t, wb)).max() <= 1e-12, (group, b)
                ref = oracle.weighting(Xb, t)
                assert abs(Ms[b] - ref.M) / abs(ref.M) <= 1e-10
            res[group] = w
        assert np.abs(res[1] - res[2]).max() <= 1e-10 * np.abs(res[2]).max()
    finally:
        mag.tune_batch_group(max(len(c) for c in clouds), 0)


def test_autotune_batch_and_table_file(mag, tmp_path):
    clouds = W.mixture_clouds(B=8, m=3, seed=21, n_lo=1000, n_hi=3000)
    X, offs = W.pack_clouds(clouds)
    ts = [40.0] * len(clouds)
    group, ms = mag.autotune_batch(dev(X), offs, ts, reps=2)
    print(f"batched factor of 8 clouds (n <= {max(len(c) for c in clouds)}): single {ms[0]:.2f} ms, "
          f"pairs {ms[1]:.2f} ms -> group {group}")
    assert group in (1, 2) and all(v > 0 for v in ms)
    assert group == (1 if ms[0] < ms[1] else 2)
    path = str(tmp_path / "tune.json")
    mag.tune_save(path)
    text = open(path).read()
    assert '"batch_group"' in text and f": {group}" in text
    nmax = max(len(c) for c in clouds)
    mag.tune_batch_group(nmax, 0)
    mag.tune_load(path)
    # the tuned grouping solves the batch to the same acceptance
    w, Ms, infos = mag.weighting_batch(dev(X), offs, ts)
    w = w.cpu().numpy()
    for b in (0, len(clouds) - 1):
        assert np.abs(oracle.residual(clouds[b], ts[b], w[offs[b]:offs[b + 1]])).max() <= 1e-12
    mag.tune_batch_group(nmax, 0)
    with pytest.raises(mag.MagError):
        mag.tune_batch_group(nmax, 3)
