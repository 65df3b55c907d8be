"""Serving through the C ABI: resident cameras, queued requests, continuous
batching across resolutions; every served view equals the same view computed
alone by ffv_interpolate, bit for bit."""
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
