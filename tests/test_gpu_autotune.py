"""Conv tile autotuning through the C ABI: the tuned net computes the same
views as the untuned one (tile choices change only the work split), and a
saved tuning table loads back into another net with the same effect."""
import pytest
import torch

from synth import scenes

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_autotune_same_result_and_roundtrip(random_weights_file, tmp_path, precision):
    from paper_2112_10603_amd import Net
    print(f"case autotune {precision}", flush=True)
    arc = scenes.camera_arc(71, 80, 112, 3, 64, (3.0, 8.0), 4.0, 0.01).to(DEV)
    pairs = [(arc[0].contiguous(), arc[1].contiguous()), (arc[1].contiguous(), arc[2].contiguous())]
    ts = [0.25, 0.75]
    plain = Net(random_weights_file, precision, 0)
    ref = plain.interpolate(pairs, ts)
    tuned = Net(random_weights_file, precision, 0)
    out = torch.empty_like(ref)
    n = tuned.autotune(pairs, ts, out)
    print(f"  tuned {n} launch shapes", flush=True)
    assert n > 10
    assert torch.equal(out, ref)  # the autotune call's own output
    assert torch.equal(tuned.interpolate(pairs, ts), ref)
    path = str(tmp_path / "tune.txt")
    tuned.save_tuning(path)
    lines = [l for l in open(path) if not l.startswith("#")]
    assert len(lines) == n
    other = Net(random_weights_file, precision, 0)
    assert other.load_tuning(path) == n
    assert torch.equal(other.interpolate(pairs, ts), ref)
    for net in (plain, tuned, other):
        net.close()


def test_load_tuning_rejects_bad_files(random_weights_file, tmp_path):
    from paper_2112_10603_amd import Net
    from paper_2112_10603_amd.ffv import FfvError
    print("case autotune bad files", flush=True)
    net = Net(random_weights_file, "bf16", 0)
    bad = {
        "garbage": "vib2.conv3 0 68 120\n",
        "unknown_layer": "vib9.conv3 0 68 120 1 256 16\n",
        "bad_tile": "vib2.conv3 0 68 120 1 48 16\n",
        "bad_width": "vib2.conv3 0 68 120 1 256 12\n",
    }
    for name, text in bad.items():
        p = tmp_path / f"{name}.txt"
        p.write_text(text)
        with pytest.raises(FfvError):
            net.load_tuning(str(p))
    with pytest.raises(FfvError):
        net.load_tuning(str(tmp_path / "missing.txt"))
    net.close()
