"""hipGraph replay of ffv_interpolate: every replay of a captured shape, with
new images, phases and output buffers and with other device work in between,
equals the eager launch sequence bit for bit (same kernels, same order)."""
import numpy as np
import pytest
import torch

from synth import scenes

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _pairs(arc):
    return [(arc[i].contiguous(), arc[i + 1].contiguous()) for i in range(arc.shape[0] - 1)]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_graph_replays_equal_eager(random_weights_file, precision):
    from paper_2112_10603_amd import Net
    print(f"case graph replay {precision}", flush=True)
    g = Net(random_weights_file, precision, 0, graphs=True)
    e = Net(random_weights_file, precision, 0, graphs=False)
    arcs = {
        "a": scenes.camera_arc(61, 48, 80, 3, 64, (3.0, 8.0), 4.0, 0.01).to(DEV),
        "b": scenes.camera_arc(62, 48, 80, 3, 64, (3.0, 8.0), 4.0, 0.01).to(DEV),
        "c": scenes.camera_arc(63, 40, 72, 2, 64, (3.0, 8.0), 4.0, 0.01).to(DEV),
    }
    rng = np.random.default_rng(3)
    # shape 1 (48x80, 3 cameras, 2 pairs x 2 phases) three times with
    # different inputs, phases and outputs; a second shape in between
    plan = ["a", "b", "c", "a", "b", "c", "a"]
    for k, name in enumerate(plan):
        arc = arcs[name]
        ts = [float(x) for x in rng.uniform(0, 1, 2)]
        got = g.interpolate(_pairs(arc), ts)
        # unrelated device work between replays
        junk = torch.randn(1 << 20, device=DEV).mul_(2.0).sum()
        ref = e.interpolate(_pairs(arc), ts)
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        diff = (got - ref).abs().max().item()
        print(f"  call {k} ({name}, t={ts[0]:.3f},{ts[1]:.3f}): max |graph - eager| = {diff}",
              flush=True)
        assert torch.equal(got, ref), f"call {k} ({name}) differs by {diff}"
    g.close()
    e.close()


def test_graph_with_view_chunks(random_weights_file):
    """A workspace cap that leaves room for one view at a time: the graph
    holds six chunk passes and still equals the eager run."""
    from paper_2112_10603_amd import Net
    print("case graph chunks bf16", flush=True)
    arc = scenes.camera_arc(64, 64, 96, 3, 64, (3.0, 8.0), 4.0, 0.01).to(DEV)
    ts = [0.2, 0.5, 0.9]
    cap = 1
    g = Net(random_weights_file, "bf16", 0, workspace_bytes=cap, graphs=True)
    e = Net(random_weights_file, "bf16", 0, workspace_bytes=cap, graphs=False)
    for rep in range(3):
        out_g = torch.full((2, 3, 3, 64, 96), float("nan"), device=DEV)
        g.interpolate(_pairs(arc), ts, out_g)
        ref = e.interpolate(_pairs(arc), ts)
        torch.cuda.synchronize()
        assert torch.equal(out_g, ref), f"replay {rep}"
    g.close()
    e.close()


def test_graph_profiling_matches_eager_counts(random_weights_file):
    """With profiling on, the captured graph carries event-record nodes
    around each kernel class: after replays the per-class launch counts and
    work equal the eager run's, and every class has positive time."""
    from paper_2112_10603_amd import Net
    print("case graph profiling", flush=True)
    arc = scenes.camera_arc(65, 48, 80, 3, 64, (3.0, 8.0), 4.0, 0.01).to(DEV)
    ts = [0.3, 0.6]
    stats = {}
    for mode in (True, False):
        net = Net(random_weights_file, "bf16", 0, graphs=mode)
        net.set_profiling(True)
        for _ in range(3):
            net.interpolate(_pairs(arc), ts)
        torch.cuda.synchronize()
        stats[mode] = {k: net.kernel_stats(k) for k in ("conv256", "conv", "convT", "pixel", "head")}
        net.close()
    for k in stats[True]:
        g, e = stats[True][k], stats[False][k]
        print(f"  {k}: graph {g} eager {e}", flush=True)
        assert g["launches"] == e["launches"] > 0
        assert g["work"] == pytest.approx(e["work"])
        assert g["ms"] > 0
