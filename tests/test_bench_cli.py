"""Host-side checks of bench.py that need no GPU: the one-GPU guard and the pass byte model."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_pass_bytes_match_the_layout_model():
    sys.path.insert(0, ROOT)
    import bench
    n = (256, 256, 64)
    zh = n[0] * n[1] * (n[2] + 1) * 16                     # half-spectrum Z (Nz + 1 entries per row)
    yb = n[0] * 2 * n[1] * (n[2] + 1) * 16                 # padded-y Y
    octant = (n[0] + 1) * (n[1] + 1) * (n[2] + 1) * 8      # FP64 symbol octant
    assert bench.pass_bytes("y_fwd", n, 16) == zh + yb == 204472320
    assert bench.pass_bytes("x_pass", n, 16) == 2 * yb + octant
    assert bench.pass_bytes("x_pars2", n, 16) == 2 * yb + octant


def test_site_bytes_cover_the_iteration():
    """Per-site algorithmic bytes of one FP64 iteration at 256x256x64 add up to the pass model
    (about 4.3 GB: every field read and written once per pass)."""
    sys.path.insert(0, ROOT)
    import bench
    import paper_2603_05194_amd as bec
    n = (256, 256, 64)
    per_launch = {s: bench.site_bytes(s, n, 16) for s in bec.SITES}
    launches = {"prec_y": 2, "y_fwd": 3, "p_lines": 3}
    total = sum(b * launches.get(s, 1) for s, b in per_launch.items())
    assert per_launch["control"] == per_launch["finish"] == 0
    assert per_launch["y_fwd"] == bench.pass_bytes("y_fwd", n, 16)
    assert per_launch["x_atkm"] == per_launch["x_pars2"] == bench.pass_bytes("x_pass", n, 16)
    assert 4.2e9 < total < 4.4e9
