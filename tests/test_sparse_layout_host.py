"""The sparse layout's slot image on the CPU (no GPU needed).

sparse_layout_host.cpp builds the image with the library's own compile code
and walks random texts through it the way the walk kernel reads it, against
a walk of the dense table: every state and the count of steps entering a
final state must agree. Cases: the large sparse byte DFA (uniform form,
keyed by bytes), per-state defaults (general form), a 200-byte and a
20-byte alphabet (keyed by columns, with the invalid column), five
exceptions a row, a dead state that half the rows reach on one byte, and a
table whose slots do not fit (no layout)."""
import os
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    from paper_1412_1741_amd import build as B

    lib_dir = os.path.dirname(B.LIB)
    if not os.path.exists(B.hipcc()) or not os.path.exists(B.LIB):
        pytest.skip("hipcc or the built library is not available")
    exe = str(tmp_path_factory.mktemp("sparse") / "sparse_layout_host")
    flags = [f for f in B.HIP_FLAGS if f not in ("-Wall",) and not f.startswith("--offload-arch")]
    subprocess.check_call([B.hipcc(), *flags, "-I", os.path.join(ROOT, "include"), "-I", B.CSRC,
                           os.path.join(ROOT, "tests", "sparse_layout_host.cpp"), "-o", exe,
                           "-L", lib_dir, "-lparem", f"-Wl,-rpath,{lib_dir}"], stderr=subprocess.DEVNULL)
    return exe


def run(harness, tmp_path, name, table, alphabet, start, accepting):
    path = tmp_path / f"{name}.bin"
    q, a = table.shape
    with open(path, "wb") as f:
        np.asarray([q, a, start, len(accepting)], np.uint32).tofile(f)
        np.frombuffer(bytes(alphabet), np.uint8).tofile(f)
        np.asarray(table, np.uint32).tofile(f)
        np.asarray(accepting, np.uint32).tofile(f)
    r = subprocess.run([harness, str(path)], capture_output=True, text=True, timeout=300)
    return r.returncode, r.stdout.strip()


def test_sparse_slots_walk_like_the_dense_table(harness, tmp_path):
    rng = np.random.default_rng(1741)
    big = W.sparse4096_dfa()
    rc, out = run(harness, tmp_path, "big", big.table, big.alphabet, big.start, big.accepting)
    assert rc == 0 and out.startswith("form=uniform"), out

    sym = rng.choice(256, size=64, replace=False).astype(np.uint8)
    acc = rng.choice(np.arange(1, 3000), size=16, replace=False)
    sp = W.sparse_dfa(rng, 3000, bytes(range(256)), 1, 4, acc, explicit_cols=sym)
    dflt = (np.arange(3000, dtype=np.uint32) % 97 + 1)[:, None]
    shifted = np.where(sp.table == 0, dflt, sp.table)
    rc, out = run(harness, tmp_path, "shifted", shifted, sp.alphabet, 5, sp.accepting)
    assert rc == 0 and out.startswith("form=general"), out

    a200 = bytes(np.sort(rng.choice(256, size=200, replace=False)).astype(np.uint8))
    cols = W.sparse_dfa(rng, 1500, a200, 1, 3, acc[:5] % 1500)
    cdef = (np.arange(1500, dtype=np.uint32) % 89 + 2)[:, None]
    rc, out = run(harness, tmp_path, "cols", np.where(cols.table == 0, cdef, cols.table), a200, 3, cols.accepting)
    assert rc == 0 and out.startswith("form=general"), out

    a20 = bytes(rng.choice(256, size=20, replace=False).astype(np.uint8))
    small = W.sparse_dfa(rng, 400, a20, 0, 3, rng.choice(np.arange(1, 400), size=9, replace=False))
    rc, out = run(harness, tmp_path, "small", small.table, a20, 0, small.accepting)
    assert rc == 0 and out.startswith("form=uniform"), out

    five = W.sparse_dfa(rng, 300, bytes(range(256)), 5, 5, acc[:3] % 300)
    rc, out = run(harness, tmp_path, "five", five.table, five.alphabet, 0, five.accepting)
    assert rc == 0 and out.startswith("form=uniform"), out

    # a dead state (the last row, absorbing) reached on byte 255 from half the rows
    q = 2000
    dead = np.zeros((q + 1, 256), dtype=np.uint32)
    for s in range(q):
        c = rng.choice(sym, size=2, replace=False)
        dead[s, c] = rng.integers(0, q, size=2)
    dead[np.flatnonzero(rng.random(q) < 0.5), 255] = q
    dead[q, :] = q
    rc, out = run(harness, tmp_path, "dead", dead, bytes(range(256)), 0, acc[:4] % q)
    assert rc == 0 and out.startswith("form=uniform"), out

    wide = W.sparse_dfa(rng, 2000, bytes(range(256)), 8, 16, acc[:3] % 2000)
    rc, out = run(harness, tmp_path, "wide", wide.table, wide.alphabet, 0, wide.accepting)
    assert rc == 3 and out == "no layout", out
