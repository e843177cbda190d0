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


CONCURRENT = r"""
import hashlib, threading
from paper_1005_3609_amd import api
jobs = [("square", 12, True), ("square", 11, True), ("square", 12, True), ("triangular", 11, True),
        ("square", 12, False), ("triangular", 11, False)]
ths = [threading.Thread(target=api.prepare_host, args=j[:2], kwargs=dict(normalised=j[2])) for j in jobs]
for t in ths:
    t.start()
for t in ths:
    t.join()
h = hashlib.sha256()
for lat, m, norm in sorted(set(jobs)):
    for which in ((4, 5) if norm else (0, 1)):
        for i in range(m):
            rp, cols, codes, nc = api.map_export(lat, m, which, i)
            for a in (rp, cols, codes):
                h.update(a.tobytes())
print(h.hexdigest())
"""

SERIAL = CONCURRENT.replace("for t in ths:\n    t.start()\nfor t in ths:\n    t.join()\n", "")


def test_concurrent_host_builds_match_serial_ones():
    # map sets requested at the same time from several threads (two of them
    # the same set; the library serializes the builds) equal the ones built
    # on demand one at a time
    env = dict(os.environ, PYTHONPATH=ROOT)
    outs = []
    for script in (CONCURRENT, SERIAL):
        r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr
        outs.append(r.stdout.strip())
    assert outs[0] == outs[1]
    assert SERIAL != CONCURRENT
