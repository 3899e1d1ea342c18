"""Parts of bench.py that need no GPU: more than one GPU is refused with a message and a
non-zero exit status before anything touches a device, and the roofline traffic is read from
the committed counter summary of the current kernels."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"] and "--gpus 1" in msg["error"]


def test_counter_summary_is_read_for_the_current_kernels():
    """bench.py's roofline traffic comes from the committed counter summary when it was taken on
    the current kernels; the scaled bytes per launch then lie within 1x-1.5x of the algorithmic
    bytes of the packed substitutions (158.3 MB per launch at 511^2, 8x8)."""
    import pytest

    sys.path.insert(0, ROOT)
    import bench

    sha = bench.kernel_source_sha(os.path.join(ROOT, "paper_1909_01467_amd", "csrc", "kernels.hip"), "k_chain_sym")
    assert sha is not None
    text = open(os.path.join(ROOT, "profiles", "lens2d_mixed_hbm_traffic.txt")).read()
    if f"k_chain_sym source sha256[:16] = {sha}" not in text:
        pytest.skip("the counters predate the current k_chain_sym (bench.py reports traffic null)")
    for kernel in ("k_chain_sym<CS_STAGE1>", "k_chain_sym<CS_FINAL>"):
        t = bench.counter_traffic(kernel, "lens2d")
        assert t is not None and 1.0 <= t / 158292992 <= 1.5, (kernel, t)



def test_lens3d_counter_summary_matches_the_plane_step_kernel():
    """The lens3d counter summary names the source sha of k_tile3 and the algorithmic bytes of its
    launches; while both match, bench.py reports its counter traffic, which lies within 1x-1.5x of the
    algorithmic bytes of one plane step (418.4 MB of packed complex64 tiles per launch at 95^3, 4x4
    beams, 7 fronts of data-flow levels).  Another amount of work per launch (a schedule that launches
    the kernel differently) gets no traffic."""
    import pytest

    sys.path.insert(0, ROOT)
    import bench

    sha = bench.kernel_source_sha(os.path.join(ROOT, "paper_1909_01467_amd", "csrc", "kernels3d.hip"), "k_tile3")
    assert sha is not None
    text = open(os.path.join(ROOT, "profiles", "lens3d_mixed_hbm_traffic.txt")).read()
    if f"k_tile3 source sha256[:16] = {sha}" not in text:
        pytest.skip("the counters predate the current k_tile3 (bench.py reports traffic null)")
    per_launch = 418435805
    t = bench.counter_traffic("k_tile3", "lens3d", per_launch)
    assert t is not None and 1.0 <= t / per_launch * 1.001 <= 1.5, t
    assert bench.counter_traffic("k_tile3", "lens3d", 325450070) is None   # the 9-front schedule's launches
