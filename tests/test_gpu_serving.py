"""Serving through the C ABI: resident cameras, queued requests, continuous
batching with several camera sizes in one batch (one launch per layer);
every served view equals the same view computed alone by ffv_interpolate,
bit for bit."""
import time

import numpy as np
import pytest
import torch

from synth import scenes
from synth.weights import write_weights_file

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def wfile(tmp_path_factory):
    return write_weights_file(str(tmp_path_factory.mktemp("ws") / "w.ffvw"), seed=0)


def _wait(net, tickets, timeout=60.0):
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        for tk in tickets:
            if tk in done:
                continue
            r = net.poll(tk)
            if r is not None:
                done[tk] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(done)}/{len(tickets)} done")
        time.sleep(0.002)
    return done


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_served_views_equal_alone(wfile, precision):
    from paper_2112_10603_amd import Net
    print(f"case serving mix {precision}", flush=True)
    arc_a = scenes.camera_arc(41, 64, 96, 3, 96, (3.0, 10.0), 5.0, 0.01).to(DEV)
    arc_b = scenes.camera_arc(42, 48, 80, 2, 64, (3.0, 8.0), 4.0, 0.01).to(DEV)
    served = Net(wfile, precision, 0, hbm_budget_bytes=8 << 30, tick_ms=2.0, max_batch_views=5)
    for i in range(3):
        served.register_camera(i, arc_a[i].contiguous())
    for i in range(2):
        served.register_camera(10 + i, arc_b[i].contiguous())
    rng = np.random.default_rng(7)
    reqs = []
    for k in range(23):
        if rng.random() < 0.6:
            j = int(rng.integers(0, 2))
            pair = (j, j + 1)
            shape = (3, 64, 96)
        else:
            pair = (10, 11)
            shape = (3, 48, 80)
        t = float(rng.uniform(0, 1))
        reqs.append((pair, t, torch.full(shape, -1.0, device=DEV)))
    tickets = [served.submit(p[0], p[1], t, out) for p, t, out in reqs]
    done = _wait(served, tickets)
    for tm in done.values():
        assert tm["t_submit"] <= tm["t_admit"] <= tm["t_launch"] <= tm["t_done"]
    st = served.serving_stats()
    assert st["completed"] == len(reqs) and st["queued"] == 0
    torch.cuda.synchronize()
    alone = Net(wfile, precision, 0)
    cams = {0: arc_a[0], 1: arc_a[1], 2: arc_a[2], 10: arc_b[0], 11: arc_b[1]}
    for (p, t, out) in reqs:
        ref = alone.interpolate([(cams[p[0]], cams[p[1]])], [t])[0, 0]
        assert torch.equal(out, ref), (p, t)
    alone.close()
    served.close()


def test_served_graph_replays_equal_eager(wfile):
    """Served batches replayed from captured graphs (one per slot and batch
    shape) equal the same requests served with graphs off, bit for bit, over
    three rounds with host synchronisation and eager work in between, so
    every shape is replayed several times."""
    from paper_2112_10603_amd import Net
    print("case serving graph replay", flush=True)
    arc = scenes.camera_arc(43, 64, 96, 3, 96, (3.0, 10.0), 5.0, 0.01).to(DEV)
    arc2 = scenes.camera_arc(44, 48, 80, 2, 64, (3.0, 8.0), 4.0, 0.01).to(DEV)
    nets = {g: Net(wfile, "bf16", 0, hbm_budget_bytes=8 << 30, tick_ms=2.0, max_batch_views=4, graphs=g)
            for g in (True, False)}
    for net in nets.values():
        for i in range(3):
            net.register_camera(i, arc[i].contiguous())
        for i in range(2):
            net.register_camera(10 + i, arc2[i].contiguous())
    rng = np.random.default_rng(11)
    reqs = []
    for k in range(14):
        if k % 3 == 2:
            reqs.append(((10, 11), float(rng.uniform(0, 1)), (3, 48, 80)))
        else:
            j = int(rng.integers(0, 2))
            reqs.append(((j, j + 1), float(rng.uniform(0, 1)), (3, 64, 96)))
    outs = {}
    for g, net in nets.items():
        outs[g] = []
        for rnd in range(3):
            o = [torch.full(shape, -1.0, device=DEV) for _, _, shape in reqs]
            tickets = [net.submit(p[0], p[1], t, oo) for (p, t, _), oo in zip(reqs, o)]
            _wait(net, tickets)
            torch.cuda.synchronize()
            torch.zeros(1 << 20, device=DEV).add_(1.0)  # eager work between rounds
            outs[g].append(o)
    for rnd in range(3):
        for k in range(len(reqs)):
            assert torch.equal(outs[True][rnd][k], outs[False][rnd][k]), (rnd, k)
            assert torch.equal(outs[True][rnd][k], outs[True][0][k]), (rnd, k)
    for net in nets.values():
        net.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_mixed_size_batch_one_launch(wfile, precision):
    """Eight requests of four camera sizes (even, ragged, one taller and one
    wider than the rest, so the slot's height and width come from different
    views) queued at once run as ONE batch (one launch time), twice (the
    second replays the batch's graph); every view equals the view computed
    alone, bit for bit."""
    from paper_2112_10603_amd import Net
    print(f"case serving mixed-size batch {precision}", flush=True)
    sizes = [(64, 96), (37, 53), (72, 40), (48, 80)]
    served = Net(wfile, precision, 0, hbm_budget_bytes=8 << 30, tick_ms=2.0, max_batch_views=8)
    alone = Net(wfile, precision, 0)
    cams = {}
    for k, (h, w) in enumerate(sizes):
        arc = scenes.camera_arc(50 + k, h, w, 2, max(h, w), (3.0, 9.0), 4.0, 0.01).to(DEV)
        for i in range(2):
            cams[10 * k + i] = arc[i].contiguous()
            served.register_camera(10 * k + i, cams[10 * k + i])
    rng = np.random.default_rng(9)
    order = [0, 1, 2, 3, 3, 2, 1, 0]
    reqs = [(10 * k, 10 * k + 1, float(rng.uniform(0, 1))) for k in order]
    refs = [alone.interpolate([(cams[l], cams[r])], [t])[0, 0] for l, r, t in reqs]
    for rnd in range(2):
        outs = [torch.full((3,) + sizes[k], -1.0, device=DEV) for k in order]
        tickets = served.submit_many([(l, r, t, o) for (l, r, t), o in zip(reqs, outs)])
        done = _wait(served, tickets)
        launches = {done[tk]["t_launch"] for tk in tickets}
        assert len(launches) == 1, (rnd, sorted(launches))
        torch.cuda.synchronize()
        for k, (o, ref) in enumerate(zip(outs, refs)):
            assert torch.equal(o, ref), (rnd, k, reqs[k], (o - ref).abs().max().item())
    alone.close()
    served.close()


def test_submit_many_all_or_nothing(wfile):
    from paper_2112_10603_amd import FfvError, Net
    net = Net(wfile, "bf16", 0, hbm_budget_bytes=4 << 30)
    img = torch.rand(3, 32, 32, device=DEV)
    net.register_camera(0, img)
    net.register_camera(1, img)
    outs = [torch.empty(3, 32, 32, device=DEV) for _ in range(3)]
    with pytest.raises(FfvError) as e:
        net.submit_many([(0, 1, 0.5, outs[0]), (0, 7, 0.5, outs[1]), (0, 1, 0.2, outs[2])])
    assert e.value.code == -1 and "request 1" in str(e.value)
    assert net.serving_stats()["queued"] == 0 and net.serving_stats()["admitted"] == 0
    assert net.submit_many([]) == []
    tks = net.submit_many([(0, 1, 0.5, outs[0]), (1, 0, 0.2, outs[1])])
    _wait(net, tks)
    net.close()


def test_serving_errors(wfile):
    from paper_2112_10603_amd import FfvError, Net
    net = Net(wfile, "bf16", 0, hbm_budget_bytes=4 << 30)
    img = torch.rand(3, 32, 32, device=DEV)
    net.register_camera(0, img)
    net.register_camera(1, img)
    out = torch.empty(3, 32, 32, device=DEV)
    with pytest.raises(FfvError) as e:
        net.submit(0, 5, 0.5, out)
    assert e.value.code == -1
    with pytest.raises(FfvError) as e:
        net.submit(0, 1, 1.5, out)
    assert e.value.code == -1
    with pytest.raises(FfvError) as e:
        net.poll(987654)
    assert e.value.code == -6
    tk = net.submit(0, 1, 0.5, out)
    _wait(net, [tk])
    with pytest.raises(FfvError) as e:
        net.poll(tk)  # already collected
    assert e.value.code == -6
    net.close()
    # serving off
    plain = Net(wfile, "bf16", 0)
    with pytest.raises(FfvError) as e:
        plain.register_camera(0, img)
    assert e.value.code == -7
    plain.close()
    # a budget that cannot hold one 1080p view
    tiny = Net(wfile, "bf16", 0, hbm_budget_bytes=64 << 20)
    big = torch.rand(3, 1080, 1920, device=DEV)
    with pytest.raises(FfvError) as e:
        tiny.register_camera(0, big)
        tiny.register_camera(1, big)
        tiny.submit(0, 1, 0.5, torch.empty_like(big))
    assert e.value.code == -3
    tiny.close()


def test_serving_failed_batch_reports_error(wfile):
    """A batch whose launch fails (host-side injected fault: nothing of it is
    queued on the device) reports FFV_ERR_DEVICE on each of its tickets;
    later batches run and match the view computed alone."""
    from paper_2112_10603_amd import FfvError, Net, debug_fault
    print("case serving launch fault", flush=True)
    arc = scenes.camera_arc(43, 32, 48, 2, 32, (3.0, 8.0), 3.0, 0.01).to(DEV)
    net = Net(wfile, "fp32", 0, hbm_budget_bytes=4 << 30, tick_ms=1.0)
    net.register_camera(0, arc[0].contiguous())
    net.register_camera(1, arc[1].contiguous())
    outs = [torch.full((3, 32, 48), -7.0, device=DEV) for _ in range(4)]
    debug_fault("launch:1")
    try:
        tks = [net.submit(0, 1, 0.25 * (k + 1), outs[k]) for k in range(4)]
        codes = {}
        t0 = time.time()
        while len(codes) < len(tks) and time.time() - t0 < 60:
            for k, tk in enumerate(tks):
                if k in codes:
                    continue
                try:
                    if net.poll(tk) is not None:
                        codes[k] = 0
                except FfvError as e:
                    codes[k] = e.code
            time.sleep(0.002)
    finally:
        debug_fault(None)
    assert len(codes) == 4
    assert codes[0] == -4, codes  # the first batch holds the first request
    assert all(c in (0, -4) for c in codes.values())
    torch.cuda.synchronize()
    alone = Net(wfile, "fp32", 0)
    for k in range(4):
        if codes[k] == 0:
            ref = alone.interpolate([(arc[0], arc[1])], [0.25 * (k + 1)])[0, 0]
            assert torch.equal(outs[k], ref)
        else:
            assert torch.all(outs[k] == -7.0)  # never written
    with pytest.raises(FfvError) as e:
        net.poll(tks[0])  # collected with its error
    assert e.value.code == -6
    # later requests run normally
    tk = net.submit(0, 1, 0.5, outs[0])
    _wait(net, [tk])
    assert torch.equal(outs[0], alone.interpolate([(arc[0], arc[1])], [0.5])[0, 0])
    alone.close()
    net.close()


def test_serving_camera_size_and_out_shape(wfile):
    from paper_2112_10603_amd import FfvError, Net
    net = Net(wfile, "bf16", 0, hbm_budget_bytes=4 << 30)
    a = torch.rand(3, 32, 32, device=DEV)
    net.register_camera(0, a)
    net.register_camera(1, a)
    with pytest.raises(FfvError) as e:
        net.register_camera(0, torch.rand(3, 48, 32, device=DEV))  # size change
    assert e.value.code == -1
    net.register_camera(0, torch.rand(3, 32, 32, device=DEV))  # same size: replaced
    with pytest.raises(ValueError):
        net.submit(0, 1, 0.5, torch.empty(3, 16, 16, device=DEV))
    tk = net.submit(0, 1, 0.5, torch.empty(3, 32, 32, device=DEV))
    _wait(net, [tk])
    net.close()


def test_alloc_fault_then_recover(wfile):
    """An injected allocation failure of the workspace surfaces as
    FFV_ERR_OOM; the next call allocates and runs."""
    from paper_2112_10603_amd import FfvError, Net, debug_fault
    net = Net(wfile, "fp32", 0)
    xl, xr = scenes.small_pair()
    pr = [(xl.to(DEV), xr.to(DEV))]
    debug_fault("alloc:1")
    try:
        with pytest.raises(FfvError) as e:
            net.interpolate(pr, [0.5])
        assert e.value.code == -2
    finally:
        debug_fault(None)
    out = net.interpolate(pr, [0.5])
    assert torch.isfinite(out).all()
    net.close()
