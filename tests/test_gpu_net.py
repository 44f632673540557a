"""The point-set network's GPU kernels against the FP64 reference in
oracle/net.py (same BF16 rounding points), and the seed's effect on the
exact search."""
import numpy as np
import pytest
import torch

from oracle import net as ref
from workloads import gen
from workloads.gen import Stream

pytestmark = pytest.mark.gpu


def batch(seed, B=6, n=300):
    xy, off = gen.rotated_line(B, n, seed)
    return xy, off


def test_forward_and_gradient_match_reference(gpu):
    from paper_1510_01041_amd import seednet
    params = ref.init_params(11)
    st = Stream(12, 120)
    for k in params:
        if k.startswith("b"):
            params[k] = st.uniform(params[k].size, -0.2, 0.2).reshape(params[k].shape)
    # FP32 masters, as the GPU holds them
    p32 = {k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in params.items()}
    xy, off = batch(13)
    B = len(off) - 1
    targets = st.uniform(2 * B, -1, 1).reshape(B, 2)
    net = seednet.SeedNet(seednet.pack(p32))
    pts, scale, doff = net.prepare(torch.from_numpy(xy).cuda(), off)
    grad, loss, out = net.gradient(pts, doff, torch.from_numpy(targets))
    pts_h = pts.cpu().numpy().astype(np.float64)
    sets = [pts_h[off[b]:off[b + 1]] for b in range(B)]
    # the prepared frame matches the reference normalisation (FP32 rounding)
    for b in range(B):
        r, c, s = ref.normalise(xy[off[b]:off[b + 1]])
        assert np.max(np.abs(r - sets[b])) < 1e-6
        assert np.allclose(scale[b].cpu().numpy(), [c[0], c[1], s[0], s[1]], rtol=0, atol=0)
    rl, rg, rout = ref.loss_and_grad(p32, sets, targets)
    assert np.allclose(out.cpu().numpy(), rout, rtol=1e-4, atol=1e-5)
    assert abs(float(loss.sum()) - rl) <= 1e-4 * max(rl, 1e-6)
    g = grad.cpu().numpy()
    gref = seednet.pack(rg)
    scale_g = np.abs(gref).max()
    assert np.max(np.abs(g - gref)) <= 1e-3 * scale_g, np.max(np.abs(g - gref)) / scale_g
    for k, shp in seednet.LAYOUT:
        a = seednet.unpack(g)[k]
        assert np.linalg.norm(a - rg[k]) <= 1e-3 * max(np.linalg.norm(rg[k]), 1e-6 * scale_g), k


def test_adam_step(gpu):
    from paper_1510_01041_amd import seednet
    net = seednet.SeedNet(seed=3)
    p0 = net.P.cpu().numpy().astype(np.float64)
    g = Stream(5, 50).uniform(seednet.N_PARAMS, -1, 1).astype(np.float32)
    gd = torch.from_numpy(g).cuda()
    net.adam(gd, lr=0.01)
    net.adam(gd, lr=0.01)
    m = v = np.zeros_like(p0)
    p = p0.copy()
    for t in (1, 2):
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g.astype(np.float64) ** 2
        p = p - 0.01 * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-8)
    assert np.allclose(net.P.cpu().numpy(), p, rtol=1e-5, atol=1e-6)


def test_slope_decoding(gpu):
    from paper_1510_01041_amd import seednet
    net = seednet.SeedNet(seed=4)
    xy, off = batch(14, B=5, n=200)
    th = net.predict_slopes(torch.from_numpy(xy).cuda(), off).cpu().numpy()
    pts, scale, doff = net.prepare(torch.from_numpy(xy).cuda(), off)
    out, _ = net.forward(pts, doff)
    o = out.cpu().numpy().astype(np.float64)
    sc = scale.cpu().numpy()
    want = np.tan(0.5 * np.arctan2(o[:, 1], o[:, 0])) * sc[:, 3] / sc[:, 2]
    assert np.allclose(th, want, rtol=1e-9)


def test_training_reduces_loss(gpu):
    from paper_1510_01041_amd import seednet, train_seednet
    net, hist = train_seednet.train(n_sets=512, n=256, epochs=6, batch=64, lr=3e-3, seed=21,
                                    chunk=256, log=print)
    assert hist["loss"][-1] < 0.7 * hist["loss"][0], hist["loss"]


def test_seed_slope_keeps_result_exact(gpu):
    """Whatever the network predicts, the search result is unchanged."""
    from paper_1510_01041_amd import seednet
    net = seednet.SeedNet(seed=9)  # untrained: arbitrary slopes
    for name, s in (("c1", 101), ("c1", 102)):
        xy = gen.make(name, s)
        d = torch.from_numpy(xy).cuda()
        th = net.predict_slopes(d, np.array([0, len(xy)]))
        a = gpu.solve(d)
        b = gpu.solve(d, seed_pairs=0, seed_theta=th)
        assert (a.width, a.theta1, a.z_lo) == (b.width, b.theta1, b.z_lo)


def test_inference_matches_reference_and_forward(gpu):
    """lms_net_infer (features pooled over many workgroups; sets above 2048
    points read strided, frame from the whole set) against the FP64 reference
    of the same inference, and bit for bit against the one-block forward pass
    on the same framed points."""
    from paper_1510_01041_amd import seednet
    from workloads.gen import planted
    params = ref.init_params(15)
    st = Stream(16, 160)
    for k in params:
        if k.startswith("b"):
            params[k] = st.uniform(params[k].size, -0.2, 0.2).reshape(params[k].shape)
    p32 = {k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in params.items()}
    net = seednet.SeedNet(seednet.pack(p32))
    sets = [planted(5000, 0.4, 77), planted(300, 0.4, 78), planted(2048, 0.45, 79),
            planted(16384, 0.45, 80)]
    off = np.concatenate([[0], np.cumsum([len(a) for a in sets])])
    xy = np.concatenate(sets)
    d = torch.from_numpy(xy).cuda()
    out = torch.empty((len(sets), 2), dtype=torch.float32, device="cuda:0")
    th = net.predict_slopes(d, off, out=out).cpu().numpy()
    o = out.cpu().numpy().astype(np.float64)
    for b, a in enumerate(sets):
        ro, rth = ref.predict(p32, a)
        assert np.allclose(o[b], ro, rtol=1e-4, atol=1e-5), (b, o[b], ro)
        assert abs(np.arctan(th[b]) - np.arctan(rth)) < 1e-3, (b, th[b], rth)
    # small sets: the same as prepare + one-block forward, bit for bit
    small = np.array([0, 300, 300 + 2048])
    xs = np.concatenate([sets[1], sets[2]])
    ds = torch.from_numpy(xs).cuda()
    out2 = torch.empty((2, 2), dtype=torch.float32, device="cuda:0")
    net.predict_slopes(ds, small, out=out2)
    pts, scale, doff = net.prepare(ds, small)
    fo, _ = net.forward(pts, doff, want_g=False)
    assert torch.equal(out2, fo)


def test_network_inside_the_solve(gpu):
    """opt.d_net_params runs the network inside lms_solve: the same as passing
    its slope as the device seed slope, and the exact answer either way."""
    from paper_1510_01041_amd import seednet
    from workloads.gen import planted
    net = seednet.SeedNet(seed=7)
    for xy in (gen.make("c1", 101), planted(3000, 0.45, 81), planted(9000, 0.45, 82)):
        d = torch.from_numpy(xy).cuda()
        th = net.predict_slopes(d, np.array([0, len(xy)]))
        a = gpu.solve(d, seed_pairs=0, net_params=net.P, window_pairs=63)
        b = gpu.solve(d, seed_pairs=0, seed_theta=th, window_pairs=63)
        c = gpu.solve(d)
        assert (a.width, a.theta1, a.z_lo, a.survivors, a.band_pass, a.bin_pass) == \
               (b.width, b.theta1, b.z_lo, b.survivors, b.band_pass, b.bin_pass)
        assert (a.width, a.theta1, a.z_lo) == (c.width, c.theta1, c.z_lo)
        g = gpu.parse(gpu.solve_async(d, 0, seed_pairs=0, net_params=net.P, graph=True))
        assert (g.width, g.theta1, g.z_lo) == (c.width, c.theta1, c.z_lo)
    with pytest.raises(gpu.LmsError):
        gpu.solve(d, net_params=net.P, seed_theta=th)


@pytest.mark.parametrize("name", ["c2", "c3a"])
def test_trained_network_prunes(gpu, name):
    """The committed network as the only source of the bound (no random seed
    pairs): its slope, computed inside the solve, then two rounds of 63 pairs
    drawn from the narrowest window found (window pairs). Against no seed at
    all (only the extreme-x pair) it must cut the pairs that pass the FP32
    band test by at least 100 times, with the same exact line. The slope alone
    (no window pairs) is reported beside it."""
    import os
    from paper_1510_01041_amd import seednet
    wpath = os.path.join(os.path.dirname(seednet.__file__), "seednet_weights.npy")
    net = seednet.SeedNet.load_weights(wpath)
    xy = gen.make(name)
    d = torch.from_numpy(xy).cuda()
    ref = gpu.solve(d)
    learned = gpu.solve(d, seed_pairs=0, net_params=net.P, window_pairs=63)
    slope_only = gpu.solve(d, seed_pairs=0, net_params=net.P)
    none = gpu.solve(d, seed_pairs=0)
    th = float(net.predict_slopes(d, np.array([0, len(xy)]))[0])
    err = abs(np.degrees(np.arctan(th) - np.arctan(ref.theta1)))
    print(name, "angle error", err, "band_pass learned", learned.band_pass, "slope only",
          slope_only.band_pass, "none", none.band_pass, flush=True)
    for r in (learned, slope_only, none):
        assert (r.width, r.theta1, r.z_lo, r.z_hi) == (ref.width, ref.theta1, ref.z_lo, ref.z_hi)
    assert err < 15.0
    assert none.band_pass >= 100 * max(learned.band_pass, 1)
