"""The CPU oracle and the library's host-side entry points built with
AddressSanitizer and UndefinedBehaviorSanitizer (no GPU): every oracle entry
point on small closed, quintic and infinite filament sets, and the parameter
derivation over valid and invalid inputs.  Any sanitizer report fails the
run (-fno-sanitize-recover)."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from paper_2406_07366_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")


def write_sets(path, sets):
    with open(path, "wb") as f:
        f.write(struct.pack("<q", len(sets)))
        for fs, order in sets:
            per = getattr(fs, "periods", None)
            f.write(struct.pack("<qqq", fs.n_fil, order, 0 if per is None else 1))
            f.write(np.ascontiguousarray(fs.offsets, dtype="<i8").tobytes())
            f.write(np.ascontiguousarray(fs.xyz, dtype="<f8").tobytes())
            f.write(np.ascontiguousarray(fs.gamma, dtype="<f8").tobytes())
            f.write(struct.pack("<ddd", fs.L, fs.a, fs.delta))
            if per is not None:
                f.write(np.ascontiguousarray(per, dtype="<i8").tobytes())


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = tmp_path / "oracle_san"
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp"] + SAN +
                   [os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_driver.c"),
                    "-o", str(exe), "-lm"], check=True)
    sets = [(W.ring(n_nodes=24), 4), (W.ring(n_nodes=24), 6),
            (W.ringpairs(npairs=2, nbg=1, seed=3), 4),
            (W.six_lines(n_per=16), 4), (W.helices(n_per=16), 6)]
    inp = tmp_path / "sets.bin"
    write_sets(inp, sets)
    r = subprocess.run([str(exe), str(inp)], capture_output=True, text=True, env=ENV,
                       timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0 and "runtime error" not in r.stderr and "ERROR" not in r.stderr
    assert r.stdout.count("set ") == 4 * len(sets) and "helpers" in r.stdout


CLANG = "/opt/rocm/llvm/bin/clang"


@pytest.mark.skipif(shutil.which("hipcc") is None or not os.path.exists(CLANG),
                    reason="no hipcc / clang")
def test_host_abi_under_address_and_undefined_sanitizers(tmp_path):
    """Every library source built with the sanitizers on the host pass (the
    device code as usual), and a C program (built by the same compiler, so
    that one sanitizer runtime serves both) over the host-side calls."""
    srcs = sorted(f for f in os.listdir(os.path.join(ROOT, "paper_2406_07366_amd", "csrc"))
                  if f.endswith(".hip"))
    host_san = []
    for flag in SAN:
        host_san += ["-Xarch_host", flag]
    procs = []
    for s in srcs:
        procs.append(subprocess.Popen(
            ["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17"] + host_san +
            ["-I", os.path.join(ROOT, "include"),
             "-I", os.path.join(ROOT, "paper_2406_07366_amd", "csrc"), "-c",
             os.path.join(ROOT, "paper_2406_07366_amd", "csrc", s),
             "-o", str(tmp_path / (s + ".o"))],
            stdout=subprocess.PIPE, stderr=subprocess.PIPE))
    for p in procs:
        _, err = p.communicate(timeout=900)
        assert p.returncode == 0, err.decode()[-2000:]
    lib = tmp_path / "libbs_san.so"
    subprocess.run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC"] + host_san +
                   ["-o", str(lib)] + [str(tmp_path / (s + ".o")) for s in srcs] + ["-lhipfft"],
                   check=True)
    exe = tmp_path / "abi_san"
    subprocess.run([CLANG, "-std=c99", "-g"] + SAN + ["-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "abi_driver.c"), "-o", str(exe), str(lib),
                    "-Wl,-rpath," + str(tmp_path)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=ENV, timeout=600)
    print(r.stdout, r.stderr[-4000:])
    assert r.returncode == 0 and "runtime error" not in r.stderr and "ERROR" not in r.stderr
    assert "0 inconsistent" in r.stdout
