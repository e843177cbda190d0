"""The factor maps do not depend on how many host threads build them (the
assembly scatters entries through atomic row cursors and sorts each row
afterwards; the reader order sorts by first reader)."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import hashlib
from paper_1005_3609_amd import api
h = hashlib.sha256()
for lat in ("square", "triangular"):
    m = 13                     # state spaces past the serial cut-off of 4096 rows
    for which in (0, 1, 2, 4, 5):
        n = m if which != 2 else len(range(0, m, 2))
        for i in range(n):
            rp, cols, codes, nc = api.map_export(lat, m, which, i)
            for a in (rp, cols, codes):
                h.update(a.tobytes())
            h.update(str(nc).encode())
    h.update(api.code_table(lat, m, normalised=True).tobytes())
print(h.hexdigest())
"""


def _digest(threads):
    env = dict(os.environ, CHROMSTRIP_THREADS=str(threads), PYTHONPATH=ROOT)
    out = subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr
    return out.stdout.strip()


def test_maps_identical_for_any_thread_count():
    assert _digest(1) == _digest(3) == _digest(8)
