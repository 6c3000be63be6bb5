"""Run-time settings of the library read from the environment (RPYW_TILE,
RPYW_RHS_WIDTH, RPYW_LOG, RPYW_AUTOTUNE_CACHE), checked in fresh processes
(the library reads them once).  No GPU needed: shape lookups are host code;
without a GPU the library reports the architecture as "unknown", so the
cache file below carries entries for both "unknown" and "gfx950"."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = """
import sys
sys.path.insert(0, {root!r})
from paper_1709_02410_amd import rpywall as rp
for prec, N, k in {queries!r}:
    print(prec, N, k, rp.get_shape(prec, N, k), flush=True)
"""


def _run(env_extra, queries):
    if not os.path.exists(os.path.join(ROOT, "paper_1709_02410_amd", "librpywall.so")):
        pytest.skip("librpywall.so not built")
    env = {k: v for k, v in os.environ.items() if not k.startswith("RPYW_")}
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", PROBE.format(root=ROOT, queries=queries)], env=env,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    shapes = [eval(line.split(" ", 3)[3]) for line in r.stdout.strip().splitlines()]
    return shapes, r.stderr


def test_tile_and_rhs_width_overrides():
    base, _ = _run({}, [(1, 50000, 16), (0, 3000, 1)])
    assert base[0]["tile"] == 64 and base[0]["kblk"] == 16
    got, _ = _run({"RPYW_TILE": "256", "RPYW_RHS_WIDTH": "4"}, [(1, 50000, 16), (0, 3000, 1)])
    assert got[0]["tile"] == 256 and got[0]["kblk"] == 4
    assert got[1]["tile"] == 256 and got[1]["kblk"] == 4
    # widths above 4 leave the symmetric kernel (which takes at most 4)
    got, _ = _run({"RPYW_RHS_WIDTH": "8"}, [(1, 3000, 1)])
    assert got[0]["kblk"] == 8 and got[0]["sym"] == 0


def test_invalid_values_are_ignored_and_logged():
    base, _ = _run({}, [(1, 50000, 16)])
    got, err = _run({"RPYW_TILE": "100", "RPYW_RHS_WIDTH": "3", "RPYW_LOG": "1"}, [(1, 50000, 16)])
    assert got == base
    assert "ignoring RPYW_TILE" in err and "ignoring RPYW_RHS_WIDTH" in err


def test_autotune_cache_is_read(tmp_path):
    path = tmp_path / "shapes.json"
    shape = {"tpl": 2, "tile": 64, "kblk": 2, "sym": 0, "ipw": 3}
    entries = [dict(arch=a, precision=1, size_class=12, k=2, **shape) for a in ("unknown", "gfx950")]
    entries.append(dict(arch="gfx000", precision=1, size_class=12, k=2, tpl=1, tile=256, kblk=1, sym=1, ipw=1))
    path.write_text(json.dumps({"version": 1, "entries": entries}))
    got, err = _run({"RPYW_AUTOTUNE_CACHE": str(path), "RPYW_LOG": "1"}, [(1, 5000, 2), (1, 9000, 2), (0, 5000, 2)])
    assert got[0] == dict(shape, mat=0)  # size class 12 = [4096, 8192), two right-hand sides; no "mat": 0
    assert got[1] != shape and got[2] != shape  # other size class, other precision
    assert "1 shapes for" in err


def test_missing_cache_is_reported_not_fatal(tmp_path):
    got, err = _run({"RPYW_AUTOTUNE_CACHE": str(tmp_path / "absent.json"), "RPYW_LOG": "1"}, [(1, 5000, 1)])
    assert got and "not read" in err


OVERRIDE_PROBE = """
import sys
sys.path.insert(0, {root!r})
from paper_1709_02410_amd import rpywall as rp
print(rp.get_shape(1, 5000, 2), flush=True)
rp.set_shape(1, 5000, 2, tpl=1, tile=256, kblk=1, sym=1, ipw=2)
print(rp.get_shape(1, 5000, 2), flush=True)
rp.reset_shape(1, 5000, 2)
print(rp.get_shape(1, 5000, 2), flush=True)
"""


def test_override_and_reset_keep_the_tuned_shape(tmp_path):
    """rpy_wall_set_shape fixes a shape over the tuned one; removing the
    override goes back to the tuned shape (here from the cache file), not to
    the built-in default."""
    if not os.path.exists(os.path.join(ROOT, "paper_1709_02410_amd", "librpywall.so")):
        pytest.skip("librpywall.so not built")
    path = tmp_path / "shapes.json"
    tuned = {"tpl": 2, "tile": 64, "kblk": 2, "sym": 0, "ipw": 3, "mat": 0}
    entries = [dict(arch=a, precision=1, size_class=12, k=2, **tuned) for a in ("unknown", "gfx950")]
    path.write_text(json.dumps({"version": 1, "entries": entries}))
    env = {k: v for k, v in os.environ.items() if not k.startswith("RPYW_")}
    env["RPYW_AUTOTUNE_CACHE"] = str(path)
    r = subprocess.run([sys.executable, "-c", OVERRIDE_PROBE.format(root=ROOT)], env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    got = [eval(line) for line in r.stdout.strip().splitlines()]
    assert got[0] == tuned
    assert got[1] == dict(tpl=1, tile=256, kblk=1, sym=1, ipw=2, mat=0)
    assert got[2] == tuned
