"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (g++), run in a child
process on tiny corpora of both symbol widths and both frequencies, chains with ties, empty and
short sequences, featurize and argument errors: no sanitizer report, and the same tables as the
plain build."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import json, sys, random
import numpy as np
sys.path.insert(0, sys.argv[1])
import gen, oracle
out = []
rng = random.Random(5)
for trial in range(24):
    bits = 8 if trial % 2 == 0 else 2
    occ = (trial // 2) % 2
    m = rng.randint(0, 6)
    sigma = rng.choice([2, 3, 4] if bits == 2 else [2, 5, 256])
    files = [bytes(rng.randrange(sigma) for _ in range(rng.choice([0, 1, 3, rng.randint(0, 50)]))) for _ in range(m)]
    corpus = gen.from_files(files, bits)
    o = oracle.Oracle(bits, oracle.FREQ_OCC if occ else oracle.FREQ_DOC, nthreads=rng.choice([1, 3]),
                      lib_path=sys.argv[2])
    o.load(corpus)
    rec = []
    for n in range(1, rng.randint(2, 9 if bits == 8 else 30)):
        rc = o.pass_(n, rng.choice([1, 3, 1000]))
        keys, counts = o.topk() if rc == 0 else (np.zeros((0, 2), np.uint64), np.zeros(0, np.uint64))
        rec.append([rc, keys.tolist(), counts.tolist()])
    if files:
        ip, ind = o.featurize(corpus)
        rec.append([ip.tolist(), ind.tolist()])
    rec.append([o.pass_(0, 5), o.pass_(1, 0)])
    out.append(rec)
print(json.dumps(out))
'''


def _run(lib, env=None):
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, lib], capture_output=True, text=True, env=env, timeout=600)
    return r


def test_oracle_under_asan_and_ubsan(tmp_path):
    libasan = subprocess.check_output(["g++", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(libasan):
        pytest.skip("no AddressSanitizer runtime for g++")
    plain = str(tmp_path / "plain.so")
    san = str(tmp_path / "san.so")
    oracle.build(force=True, out=plain)
    oracle.build(force=True, out=san, flags=["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                                            "-fno-omit-frame-pointer", "-g"])
    env = dict(os.environ, LD_PRELOAD=libasan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    a = _run(plain)
    assert a.returncode == 0, a.stderr[-2000:]
    b = _run(san, env)
    assert b.returncode == 0, b.stderr[-4000:]
    assert "runtime error" not in b.stderr and "AddressSanitizer" not in b.stderr, b.stderr[-4000:]
    assert json.loads(a.stdout) == json.loads(b.stdout)


LIB_CHILD = r'''
import sys
sys.path.insert(0, sys.argv[1])
import paper_2511_14955_amd as ig
lib = ig.load_library()
missing = [f for f in ig.header_functions() if not hasattr(lib, f)]
assert not missing, missing
try:
    ig.Intergrams()
    print("created")
except ig.IGError as e:          # no GPU here: the create path fails cleanly
    print("create failed", e.code)
print(lib.ig_last_error(None).decode())
'''


def test_library_host_code_under_asan():
    """The host side of libintergrams.so built with AddressSanitizer and UndefinedBehaviorSanitizer
    loads, exports every declared call and runs its context set-up path (which on a machine
    without a GPU ends in IG_EDEVICE) without a sanitizer report."""
    from paper_2511_14955_amd import build
    rt = build.sanitizer_runtime()
    if not rt:
        pytest.skip("no sanitizer runtime for hipcc")
    so = build.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=rt, IG_LIBRARY=so, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", LIB_CHILD, ROOT], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "created" in r.stdout or "create failed" in r.stdout
