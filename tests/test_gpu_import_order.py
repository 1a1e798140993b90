"""The binding works in a fresh interpreter that never imported torch itself:
it must load the HIP runtime torch uses before the library (two runtimes in
one process make the library's first device allocation fail)."""

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = """
from paper_2403_11156_amd import scenes, sph
sc = scenes.small_scene(6, 5, 4)
sim = sph.Simulation(sc)
sim.build_neighbors()
st = sim.step()
assert st["dt"] > 0
sim.close()
print("binding ok", flush=True)
"""


def test_binding_without_torch_imported_first():
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, capture_output=True, text=True, timeout=300)
    print(r.stdout, r.stderr[-2000:], flush=True)
    assert r.returncode == 0 and "binding ok" in r.stdout
