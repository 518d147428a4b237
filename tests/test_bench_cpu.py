"""Host logic of bench.py, without a GPU: the one-GPU guard, the reading of
the committed counter summary, the kernel-source digest that keys it, and
the flop accounting from a launch's census."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_is_read_only_for_the_profiled_source_and_shape(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "k_nav_tiles_batched512.md").write_text(
        "# summary\n\ntraffic: kernel_source=abcdef0123456789 launch=4,0 bytes_per_launch=387000000\n"
        "traffic: kernel_source=abcdef0123456789 launch=2,0 bytes_per_launch=322000000\n"
        "traffic: kernel_source=1111111111111111 launch=4,0 bytes_per_launch=1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_traffic("abcdef0123456789", "4,0") == 387e6
    assert bench.read_traffic("abcdef0123456789", "2,0") == 322e6
    assert bench.read_traffic("abcdef0123456789", "3,1") is None
    assert bench.read_traffic("0" * 16, "4,0") is None
    (tmp_path / "profiles" / "k_nav_tiles_batched512.md").unlink()
    assert bench.read_traffic("abcdef0123456789", "4,0") is None


def test_committed_summary_names_a_digest_and_the_default_shape():
    path = os.path.join(ROOT, "profiles", "k_nav_tiles_batched512.md")
    lines = [ln.split() for ln in open(path) if ln.startswith("traffic:")]
    shapes = {dict(kv.split("=", 1) for kv in ln[1:])["launch"] for ln in lines}
    assert "4,0" in shapes                                        # the autotuned launch shape
    for ln in lines:
        vals = dict(kv.split("=", 1) for kv in ln[1:])
        assert len(vals["kernel_source"]) == 16
        assert 255e6 < float(vals["bytes_per_launch"]) < 1e9   # at least the algorithmic 255.5 MB
    valu = [dict(kv.split("=", 1) for kv in ln.split()[1:]) for ln in open(path) if ln.startswith("valu:")]
    assert {v["launch"] for v in valu} >= {"4,0", "4,0,nocull"}
    for v in valu:
        assert 0 < float(v["f64_per_launch"]) < float(v["valu_per_launch"])


def test_profile_figures_are_read_for_their_source_only(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "k_nav_tiles_batched512.md").write_text(
        "valu: kernel_source=abcdef0123456789 launch=4,0 valu_per_launch=100 f64_per_launch=40\n"
        "valu: kernel_source=abcdef0123456789 launch=4,0,nocull valu_per_launch=900 f64_per_launch=500\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_profile("valu", "abcdef0123456789", "4,0", "f64_per_launch") == 40
    assert bench.read_profile("valu", "abcdef0123456789", "4,0,nocull", "valu_per_launch") == 900
    assert bench.read_profile("valu", "abcdef0123456789", "2,0", "f64_per_launch") is None
    assert bench.read_profile("valu", "0" * 16, "4,0", "f64_per_launch") is None
    assert bench.read_profile("traffic", "abcdef0123456789", "4,0", "bytes_per_launch") is None


def test_digest_ignores_comments_and_layout_only(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_1312_0816_amd", "csrc")
    dst = tmp_path / "paper_1312_0816_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in ("geonav_device.hpp", "geonav_kernels.hip"):
        shutil.copy(os.path.join(src, f), dst / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.kernel_source_digest()
    p = dst / "geonav_kernels.hip"
    text = p.read_text()
    # comments added, every line break doubled and indented further
    p.write_text("// a comment\n/* and a\n   block */\n" + text.replace("\n", "\n\n  "))
    assert bench.kernel_source_digest() == d0
    # one declaration more
    p.write_text(text + "\nint x;\n")
    assert bench.kernel_source_digest() != d0


def test_census_flops_by_hand():
    from paper_1312_0816_amd import geonav as gv
    counts = [0] * gv.CENSUS_SLOTS
    counts[gv.CENSUS_TRACKS] = 10
    counts[gv.CENSUS_CULL] = 100
    counts[0] = 5       # box daughters evaluated
    counts[5] = 3       # cones with an inner nappe
    per_eval = bench.FLOPS_ROTATION + 3
    want = (10 * (bench.FLOPS_MOTHER_BOX + bench.FLOPS_TRACK_CULL) + 100 * bench.FLOPS_CULL_TEST
            + 5 * (per_eval + bench.FLOPS_DIST_OUT[0]) + 3 * (per_eval + bench.FLOPS_DIST_OUT[5]))
    assert bench.census_flops(counts, True) == want
    # without culling: no per-track culling constants
    assert bench.census_flops(counts, False) == want - 10 * bench.FLOPS_TRACK_CULL


@pytest.mark.parametrize("sections", [2.0, 4.0])
def test_polycone_flops_grow_with_sections(sections):
    assert bench.pcon_flops(sections + 1, False, False) > bench.pcon_flops(sections, False, False)
    assert bench.pcon_flops(sections, True, False) > bench.pcon_flops(sections, False, False)
    assert bench.pcon_flops(sections, False, True) > bench.pcon_flops(sections, False, False)
