"""GPU parity of the learned warm start: histograms, the network's FP32 and
BF16 forward, its gradient and Adam steps against the FP64 oracle, the
start post-processing, the fall-back rule, and the gain of a trained network
over the evenly spaced start."""
import numpy as np
import pytest

from oracle import fcm_hist, mlp_ref
from phantom import PhantomParams, jittered_params, phantom

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1601_00072_amd import _lib
    _lib.load()
    return torch, torch.device("cuda:0")


def announce(*what):
    print("CASE", *what, flush=True)


def rand_hists(rng, B):
    """Histogram-like inputs: sparse non-negative rows summing to 1."""
    h = rng.gamma(0.3, 1.0, size=(B, 256)) * (rng.random((B, 256)) < 0.6)
    h[:, 0] += 1e-3
    return h / h.sum(axis=1, keepdims=True)


def dev(torch_dev, a, dtype=None):
    torch, d = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype or np.float32)).to(d)


def test_histogram_matches_bincount(torch_dev):
    torch, d = torch_dev
    from paper_1601_00072_amd import histogram
    announce("histogram")
    rng = np.random.default_rng(1)
    sizes = [1, 15, 16, 17, 4095, 65536, 100003, 3, 2 ** 20 + 7]
    parts = [rng.integers(0, 256, size=s, dtype=np.uint8) for s in sizes]
    parts[6][:] = 7                                       # a constant instance
    flat = np.concatenate(parts)
    buf = torch.zeros(flat.size + 8, dtype=torch.uint8, device=d)
    buf[3:3 + flat.size] = torch.from_numpy(flat).to(d)   # unaligned start
    h = histogram(buf[3:3 + flat.size], sizes).cpu().numpy()
    for i, p in enumerate(parts):
        want = (np.bincount(p, minlength=256) / p.size).astype(np.float32)
        assert np.array_equal(h[i], want), i


@pytest.mark.parametrize("C", [3, 4, 8])
def test_forward_fp32_and_bf16_against_oracle(torch_dev, C):
    from paper_1601_00072_amd import MLP
    announce("forward C", C)
    rng = np.random.default_rng(10 + C)
    X = rand_hists(rng, 37)
    with MLP(C, seed=5) as net:
        theta = net.params().astype(np.float64)
        theta += 0.05 * rng.standard_normal(theta.size)        # non-zero biases too
        net.set_params(theta.astype(np.float32))
        theta = net.params().astype(np.float64)
        y32 = net.forward(dev(torch_dev, X)).cpu().numpy()
        y16 = net.forward(dev(torch_dev, X), bf16=True).cpu().numpy()
    ref = mlp_ref.forward(theta, X.astype(np.float32).astype(np.float64), C)[0]
    ref16 = mlp_ref.forward_bf16(theta, X.astype(np.float32).astype(np.float64), C)
    scale = 1.0 + np.abs(ref)
    e32 = float(np.max(np.abs(y32 - ref) / scale))
    e16 = float(np.max(np.abs(y16 - ref16) / scale))
    print(f"fp32 vs FP64 {e32:.2e}, bf16 vs BF16 oracle {e16:.2e}, bf16 vs FP64 "
          f"{float(np.max(np.abs(y16 - ref) / scale)):.2e}")
    # FP32: sums of at most 256 products, a few ulp of the magnitudes
    assert e32 <= 2e-5
    # BF16: the FP32 accumulation can move a hidden activation across a BF16
    # rounding boundary (one BF16 ulp, 2^-7 relative, for that activation)
    assert e16 <= 2e-3


@pytest.mark.parametrize("C,B", [(4, 64), (3, 61), (8, 200)])
def test_loss_and_gradient_against_oracle(torch_dev, C, B):
    from paper_1601_00072_amd import MLP
    announce("grad C", C, "B", B)
    rng = np.random.default_rng(100 + C + B)
    X = rand_hists(rng, B).astype(np.float32)
    T = rng.uniform(0.0, 1.0, size=(B, C)).astype(np.float32)
    with MLP(C, seed=7) as net:
        theta = net.params().astype(np.float64)
        theta += 0.02 * rng.standard_normal(theta.size)
        net.set_params(theta.astype(np.float32))
        theta = net.params().astype(np.float64)
        loss, g = net.loss_grad(dev(torch_dev, X), dev(torch_dev, T))
    Xd, Td = X.astype(np.float64), T.astype(np.float64)
    lref = mlp_ref.loss(theta, Xd, Td, C)
    gref = mlp_ref.grad(theta, Xd, Td, C)
    assert abs(loss - lref) <= 1e-5 * lref
    for (name, a, b) in zip(("W1", "b1", "W2", "b2", "W3", "b3"), mlp_ref.unpack(g.astype(np.float64), C),
                            mlp_ref.unpack(gref, C)):
        err = float(np.max(np.abs(a - b)))
        ref = float(np.max(np.abs(b)))
        print(name, f"max |dg| {err:.2e} of max |g| {ref:.2e}")
        assert err <= 1e-4 * ref + 1e-9, name


def test_adam_steps_against_oracle(torch_dev):
    """Full-batch training (one minibatch per epoch) is plain Adam on the full
    gradient; three steps against the oracle's Adam."""
    from paper_1601_00072_amd import MLP
    announce("adam")
    C, B, lr, steps = 4, 96, 1e-3, 3
    rng = np.random.default_rng(3)
    X = rand_hists(rng, B).astype(np.float32)
    T = rng.uniform(0.2, 0.8, size=(B, C)).astype(np.float32)
    with MLP(C, seed=11) as net:
        theta0 = net.params().astype(np.float64)
        losses = net.train(dev(torch_dev, X), dev(torch_dev, T), epochs=steps, batch=B, lr=lr, seed=2)
        theta_gpu = net.params().astype(np.float64)
    th, m, v = theta0.copy(), np.zeros_like(theta0), np.zeros_like(theta0)
    gmin = np.full(theta0.size, np.inf)
    ref_losses = []
    for k in range(1, steps + 1):
        ref_losses.append(mlp_ref.loss(th, X.astype(np.float64), T.astype(np.float64), C))
        g = mlp_ref.grad(th, X.astype(np.float64), T.astype(np.float64), C)
        gmin = np.minimum(gmin, np.abs(g))
        th, m, v = mlp_ref.adam_step(th, g, m, v, k, lr=lr)
    d = np.abs(theta_gpu - th)
    # every Adam step moves a parameter by at most about lr; where the
    # gradient is well above Adam's eps at every step, the steps agree closely
    assert np.all(d <= 2.0 * lr * steps)
    well = gmin > 1e-5
    assert well.mean() > 0.5
    assert float(np.max(d[well])) <= 1e-3 * lr * steps
    assert np.allclose(losses, ref_losses, rtol=1e-5)


def test_training_is_deterministic_and_reduces_loss(torch_dev):
    from paper_1601_00072_amd import MLP
    announce("train determinism")
    rng = np.random.default_rng(4)
    X = rand_hists(rng, 700).astype(np.float32)
    T = np.sort(rng.uniform(0.0, 1.0, size=(700, 4)), axis=1).astype(np.float32)
    out = []
    for _ in range(2):
        with MLP(4, seed=21) as net:
            losses = net.train(dev(torch_dev, X), dev(torch_dev, T), epochs=6, batch=128, lr=2e-3, seed=9)
            out.append((losses, net.params()))
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][0], out[1][0])
    assert out[0][0][-1] < out[0][0][0]


def post_reference(y, hist, C):
    """The start post-processing rules written out: 255 y sorted, clamped to
    the histogram's range, gaps of at least 1 (pushed up, then back from the
    top), NaN where impossible."""
    nz = np.nonzero(hist > 0)[0]
    lo, hi = int(nz.min()), int(nz.max())
    with np.errstate(invalid="ignore"):
        v = np.sort((np.float32(255.0) * np.asarray(y, dtype=np.float32)).astype(np.float32)).astype(np.float64)
    if hi - lo < C - 1 or not np.all(np.isfinite(v)):
        return np.full(C, np.nan)
    v = np.clip(v, lo, hi)
    for k in range(1, C):
        v[k] = max(v[k], v[k - 1] + 1.0)
    if v[-1] > hi:
        v[-1] = hi
        for k in range(C - 2, -1, -1):
            v[k] = min(v[k], v[k + 1] - 1.0)
    return v


def const_net(C, values):
    """A network whose output is the constant values / 255 (all weights 0)."""
    from paper_1601_00072_amd import MLP
    net = MLP(C, seed=0)
    theta = np.zeros(net.n_params, dtype=np.float32)
    theta[-C:] = np.asarray(values, dtype=np.float64) / 255.0
    net.set_params(theta)
    return net


@pytest.mark.parametrize("values,levels", [([200.0, 10.0, 90.0, 91.2], (5, 180)), ([0.0, 0.0, 0.0, 0.0], (20, 60)),
                                           ([300.0, 299.0, 298.0, 250.0], (0, 255)), ([50, 60, 70, 80], (30, 32)),
                                           ([np.nan, 60, 70, 80], (0, 255))])
def test_warm_centroid_post_processing(torch_dev, values, levels):
    from paper_1601_00072_amd import histogram
    announce("post", values, levels)
    torch, d = torch_dev
    lo, hi = levels
    x = np.repeat(np.arange(lo, hi + 1, dtype=np.uint8), 3)
    xt = torch.from_numpy(x).to(d)
    h = histogram(xt, [x.size])
    with const_net(4, values) as net:
        v0 = net.warm_centroids(h).cpu().numpy()[0]
    # all weights are zero, so the BF16 network outputs its BF16-rounded b3
    y = mlp_ref.bf16_round((np.asarray(values, dtype=np.float64) / 255.0).astype(np.float32).astype(np.float64))
    want = post_reference(y.astype(np.float32), fcm_hist.histogram(x).astype(np.float64), 4)
    assert np.array_equal(np.isnan(v0), np.isnan(want))
    assert np.allclose(v0[~np.isnan(want)], want[~np.isnan(want)], rtol=0, atol=0)


def three_level_image():
    """Grey levels 10, 128, 245 with counts 1000, 2000, 1000 and C = 2, m = 2:
    two local minima of J_m (level 128 joins the lower or the upper
    cluster); the evenly spaced start reaches the lower J_m."""
    return np.concatenate([np.full(1000, 10, np.uint8), np.full(2000, 128, np.uint8), np.full(1000, 245, np.uint8)])


def test_solve_warm_follows_algorithm_1_and_falls_back(torch_dev):
    torch, d = torch_dev
    from paper_1601_00072_amd import FCM
    announce("solve_warm policy")
    x = three_level_image()
    h = fcm_hist.histogram(x)
    xt = torch.from_numpy(x).to(d)
    plain = fcm_hist.solve(h, 2, 2.0, 1e-5, 300)
    # "same" leads to the plain start's minimum, "worse" to the other one
    starts = {"same": [20.0, 160.0], "worse": [69.0, 240.0]}
    oras = {k: fcm_hist.solve(h, 2, 2.0, 1e-5, 300, v0=np.asarray(v, np.float64)) for k, v in starts.items()}
    Jp = plain.J[plain.T]
    assert abs(oras["same"].J[oras["same"].T] - Jp) <= 1e-9 * Jp
    assert oras["worse"].J[oras["worse"].T] > Jp * (1 + 1e-3)
    for k, v in starts.items():
        with const_net(2, v) as net, FCM(xt, 2) as f:
            rw, used, rp = f.solve_warm(net, check=True)
            lab = f.labels().cpu().numpy()
            # the plain solve is the oracle's from the evenly spaced start
            assert rp.iters == plain.T and np.allclose(rp.centroids, plain.v[plain.T], rtol=1e-5)
            assert used == (k == "same")
            ref = oras[k] if used else plain
            assert rw.iters == ref.T
            assert np.allclose(rw.centroids, ref.v[ref.T], rtol=1e-5)
            assert np.array_equal(lab, fcm_hist.level_labels(ref.v[ref.T])[x])
            # without the check the warm solve is returned as it is
            rw2, used2, _ = f.solve_warm(net, check=False)
            assert used2 and rw2.iters == oras[k].T
            assert np.allclose(rw2.centroids, oras[k].v[oras[k].T], rtol=1e-5)


def test_invalid_network_output_selects_the_plain_start(torch_dev):
    torch, d = torch_dev
    from paper_1601_00072_amd import FCM
    announce("nan output")
    x = phantom(PhantomParams(shape=(90, 110), seed=31)).ravel()
    xt = torch.from_numpy(x).to(d)
    with const_net(4, [np.nan, 1, 2, 3]) as net, FCM(xt, 4) as f:
        rw, used, rp = f.solve_warm(net, check=True)
    assert used and rw.iters == rp.iters and np.array_equal(rw.centroids, rp.centroids)


def test_batch_warm_matches_single_instances(torch_dev):
    torch, d = torch_dev
    from paper_1601_00072_amd import FCM, FCMBatch
    announce("batch warm")
    xs = [phantom(jittered_params((64 + 9 * i, 70), 777 + i)).ravel() for i in range(10)]
    xs.append(three_level_image())
    Cs = [4] * 10 + [2]
    flat = torch.from_numpy(np.concatenate(xs)).to(d)
    with const_net(4, [10.0, 60.0, 100.0, 140.0]) as net:
        with FCMBatch(flat, [a.size for a in xs], [dict(n_clusters=c) for c in Cs]) as b:
            warm, used, plain = b.solve_warm(net, check=True)
        off = 0
        for i, (a, c) in enumerate(zip(xs, Cs)):
            xi = flat[off:off + a.size]
            off += a.size
            with FCM(xi, c) as f:
                if c == net.C:
                    r, u, rp = f.solve_warm(net, check=True)
                    assert u == used[i]
                else:
                    r = f.solve()
                    assert not used[i]
            # same start, same iteration: the two paths differ only in the
            # order of their FP32 partial sums
            assert abs(r.iters - warm[i].iters) <= 1, i
            if r.iters == warm[i].iters:
                assert np.max(np.abs(r.centroids - warm[i].centroids) / np.maximum(np.abs(r.centroids), 1)) <= 2e-5


def test_trained_network_gain(torch_dev):
    """Train on GPU-converged centroids of 2,000 jittered 96x96 phantoms, then
    compare on 64 held-out phantoms: the warm start must take fewer
    iterations on average, and every accepted warm result must reach the
    plain J_m within 1e-6."""
    torch, d = torch_dev
    from paper_1601_00072_amd import learn
    announce("gain")
    train = [phantom(jittered_params((96, 96), 10 ** 6 + i)).ravel() for i in range(2000)]
    held = [phantom(jittered_params((96, 96), 2 * 10 ** 6 + i)).ravel() for i in range(64)]
    x, sizes = learn.upload(train, d)
    net, losses, _, t_train = learn.train(x, sizes, C=4, epochs=60, batch=128, lr=2e-3, seed=3)
    print("training loss", losses[0], "->", losses[-1], f"({t_train:.2f} s)")
    xh, sh = learn.upload(held, d)
    ev = learn.evaluate_instances(net, xh, sh, C=4)
    print(ev)
    net.close()
    assert losses[-1] < 0.1 * losses[0]
    assert ev["iters_warm_mean"] < ev["iters_plain_mean"]
    assert ev["max_rel_J_excess_accepted"] <= 1e-6


@pytest.mark.parametrize("shape,driver,exchange", [((64, 128, 128), 2, 0), ((64, 128, 128), 1, 0), ((173, 211), 2, 0),
                                                    ((64, 128, 128), 2, 3), ((173, 211), 2, 3)])
def test_warm_start_in_kernel_and_launched(torch_dev, shape, driver, exchange):
    """The persistent driver computes the histogram and runs the network inside
    its one launch; the graph driver launches the histogram and network
    kernels first.  Both must start from the start the oracle derives (FP64
    BF16 forward + the post-processing rule) and then follow the FP64 oracle."""
    torch, d = torch_dev
    from paper_1601_00072_amd import FCM, MLP
    from tests import _parity as P
    announce("warm start", shape, "driver", driver, "exchange", exchange)
    x = phantom(PhantomParams(shape=shape, seed=17)).ravel()
    xt = torch.from_numpy(x).to(d)
    h = fcm_hist.histogram(x)
    hn = (h / x.size).astype(np.float32).astype(np.float64)
    with MLP(4, seed=3) as net:
        theta = net.params().astype(np.float64)
        y = mlp_ref.forward_bf16(theta, hn[None, :], 4)[0]
        with FCM(xt, 4) as f:
            f.set_tuning(driver=driver, exchange=exchange)
            res, used, _ = f.solve_warm(net, check=False)
            traj = P.gpu_trajectory(f, res.iters)
            lab = f.labels().cpu().numpy()
    v0 = post_reference(y.astype(np.float32), hn, 4)
    assert np.all(np.isfinite(v0))
    v0 = v0.astype(np.float32).astype(np.float64)
    # the BF16 kernel accumulates in FP32: its output can differ from the FP64
    # oracle's by a few FP32 ulp (and one BF16 step where a boundary is crossed)
    assert np.max(np.abs(traj[0][0] - v0)) <= 0.05, (traj[0][0], v0)
    ora = fcm_hist.solve(h, 4, 2.0, 1e-5, 300, v0=v0)
    if res.iters != ora.T:
        ext = fcm_hist.solve(h, 4, 2.0, 0.0, max(res.iters, ora.T) + 1, v0=ora.v[0])
        P.check_iterations(res, ora.T, ext, 1e-5, hist=h, m=2.0, gpu_vs=traj[0])
        ora = ext
    P.compare(res, traj, ora, 1e-5, hist=h, m=2.0)
    P.check_labels(x, lab, ora.v[res.iters])


def _fnv1a(data: bytes, h: int = 0xCBF29CE484222325) -> int:
    """FNV-1a 64 (Fowler, Noll and Vo), written from its published definition."""
    for b in data:
        h = ((h ^ b) * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def test_network_file_round_trip_and_rejections(torch_dev, tmp_path):
    """fcm_mlp_save / fcm_mlp_load: the documented header, bit-exact
    parameters, and every malformed file refused with the network unchanged."""
    import struct
    from paper_1601_00072_amd import MLP
    from paper_1601_00072_amd.api import FcmError
    announce("network file")
    torch, d = torch_dev
    rng = np.random.default_rng(11)
    src = MLP(4, seed=123)
    theta = rng.standard_normal(src.n_params).astype(np.float32)
    src.set_params(theta)
    path = str(tmp_path / "net.fcmmlp")
    src.save(path)
    raw = open(path, "rb").read()
    assert len(raw) == 64 + 4 * src.n_params
    magic, version, dtype, n_in, h1, h2, C, n_params, seed, layout, checksum = struct.unpack("<8sIIiiiiqQQQ", raw[:64])
    assert (magic, version, dtype, n_in, h1, h2, C, n_params, seed) == (b"FCMMLP01", 1, 0, 256, 128, 64, 4,
                                                                          src.n_params, 123)
    words = struct.pack("<8I", version, dtype, n_in, h1, h2, C, n_params & 0xFFFFFFFF, n_params >> 32)
    assert layout == _fnv1a(words)
    assert checksum == _fnv1a(raw[64:])
    assert np.array_equal(np.frombuffer(raw[64:], dtype="<f4"), theta)

    dst = MLP(4, seed=7)
    before = dst.params()
    dst.load(path)
    assert np.array_equal(dst.params(), theta)
    hist = dev(torch_dev, rand_hists(rng, 5))
    assert torch.equal(dst.forward(hist, bf16=True), src.forward(hist, bf16=True))
    dst.set_params(before)

    def expect(status, data, net=dst):
        bad = str(tmp_path / "bad.fcmmlp")
        with open(bad, "wb") as fh:
            fh.write(data)
        with pytest.raises(FcmError) as e:
            net.load(bad)
        assert e.value.status == status
        assert np.array_equal(net.params(), before if net is dst else net.params())

    flip = bytearray(raw)
    flip[64 + 4 * 1000] ^= 0x01
    expect(-7, bytes(flip))                       # checksum
    expect(-7, raw[:-4])                          # truncated
    expect(-7, raw + b"\0")                       # trailing bytes
    expect(-7, b"XCMMLP01" + raw[8:])             # magic
    expect(-7, raw[:8] + struct.pack("<I", 2) + raw[12:])   # version
    hdr = bytearray(raw)
    hdr[24:28] = struct.pack("<i", 3)             # layer sizes changed without the layout hash
    expect(-7, bytes(hdr))
    with pytest.raises(FcmError) as e:
        dst.load(str(tmp_path / "missing.fcmmlp"))
    assert e.value.status == -7
    with MLP(3, seed=0) as other:                 # a file of C = 4 into a network of C = 3
        p3 = other.params()
        with pytest.raises(FcmError) as e:
            other.load(path)
        assert e.value.status == -1
        assert np.array_equal(other.params(), p3)
    src.close()
    dst.close()


def test_batch_targets_are_sorted_centroids_over_255(torch_dev):
    torch, d = torch_dev
    from paper_1601_00072_amd import FCMBatch
    from paper_1601_00072_amd.api import FcmError
    announce("batch targets")
    xs = [phantom(jittered_params((40 + 7 * i, 50), 900 + i)).ravel() for i in range(9)]
    flat = torch.from_numpy(np.concatenate(xs)).to(d)
    with FCMBatch(flat, [a.size for a in xs], [dict(n_clusters=4)] * len(xs)) as b:
        with pytest.raises(FcmError):
            b.targets(4)                          # before a solve
        res = b.solve()
        t = b.targets(4).cpu().numpy()
        with pytest.raises(FcmError):
            b.targets(3)                          # C differs from the instances'
    want = np.stack([(np.sort(r.centroids) / 255.0).astype(np.float32) for r in res])
    assert t.dtype == np.float32 and np.array_equal(t, want)


def test_batch_warm_falls_back_per_instance(torch_dev):
    """fcm_batch_solve_warm: an instance whose warm start reaches a worse
    minimum returns its plain result (and the batch's labels are the plain
    ones), its neighbours keep their warm results."""
    torch, d = torch_dev
    from paper_1601_00072_amd import FCMBatch
    announce("batch warm fall-back")
    tri = three_level_image()
    # two noisy levels: both starts reach the same minimum (J > 0)
    rng = np.random.default_rng(5)
    two = np.clip(np.rint(np.concatenate([rng.normal(30, 6, 1500), rng.normal(200, 6, 1500)])), 0, 255).astype(np.uint8)
    xs = [two, tri, two]
    flat = torch.from_numpy(np.concatenate(xs)).to(d)
    h_tri = fcm_hist.histogram(tri)
    plain = fcm_hist.solve(h_tri, 2, 2.0, 1e-5, 300)
    worse = fcm_hist.solve(h_tri, 2, 2.0, 1e-5, 300, v0=np.array([69.0, 240.0]))
    assert worse.J[worse.T] > plain.J[plain.T] * (1 + 1e-3)
    with const_net(2, [69.0, 240.0]) as net:
        with FCMBatch(flat, [a.size for a in xs], [dict(n_clusters=2)] * 3) as b:
            warm, used, pl = b.solve_warm(net, check=True)
            lab = b.labels().cpu().numpy()
            assert list(used) == [True, False, True]
            assert warm[1].iters == pl[1].iters == plain.T
            assert np.allclose(warm[1].centroids, plain.v[plain.T], rtol=1e-5)
            off = two.size
            assert np.array_equal(lab[off:off + tri.size], fcm_hist.level_labels(plain.v[plain.T])[tri])
            for i in (0, 2):   # the same minimum from either start
                assert np.allclose(warm[i].centroids, pl[i].centroids, rtol=1e-5)
                assert abs(warm[i].J - pl[i].J) <= 1e-6 * pl[i].J
            w2, u2, p2 = b.solve_warm(net, check=False)
            assert p2 is None and list(u2) == [True, True, True]
            assert w2[1].iters == worse.T and np.allclose(w2[1].centroids, worse.v[worse.T], rtol=1e-5)
