"""AddressSanitizer and UndefinedBehaviorSanitizer builds, run on the CPU.

* The C oracle, compiled into tests/sanitize/oracle_check.c, runs every entry point on small problems of
  each kind (two-level solves in both forms, the pieces of a cycle, three levels with and without
  nested iteration, a refused argument).
* The library's host code -- argument checks and workspace layout -- is compiled host-only (no device
  code; the device code objects the host side would register are stood in for by empty arrays, which
  a run that launches nothing never reads) and driven by tests/sanitize/host_check.c.  Its workspace
  sizes and interval counts must equal those of the production library.

Any sanitizer report aborts the run (halt_on_error), and leaks are reported.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2107_09596_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_check")
        c = run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", *SAN, os.path.join(HERE, "sanitize", "oracle_check.c"),
                 "-lm", "-o", exe])
        assert c.returncode == 0, c.stderr
        r = run([exe], env=ENV)
        out = r.stdout + r.stderr
        assert r.returncode == 0 and "all checks passed" in r.stdout, out
        assert "runtime error" not in out and "AddressSanitizer" not in out, out


# (problem, options) pairs: every kind and layout branch, and configurations the library refuses
CONFIGS = [
    (dict(kind=W.HEAT1D, nx=64, nt=64), dict(m=4, k=2)),
    (dict(kind=W.HEAT1D, nx=1023, nt=1000), dict(m=16, k=3, relax=0)),
    (dict(kind=W.HEAT2D, nx=16, ny=16, nt=32), dict(m=4, k=2)),
    (dict(kind=W.HEAT2D, nx=128, ny=128, nt=4096), dict(m=32, k=13, coarse_solver=2)),
    (dict(kind=W.HEAT2D, nx=33, ny=21, nt=30), dict(m=4, k=40, coarse_solver=1)),
    (dict(kind=W.AC2D, nx=32, ny=32, nt=64), dict(m=4, k=3, coarse_substeps=2, precision=1)),
    (dict(kind=W.AC2D, nx=256, ny=256, nt=8192), dict(m=64, k=13, coarse_substeps=4, precision=1)),
    (dict(kind=W.AC2D, nx=256, ny=256, nt=256), dict(m=8, k=2, coarse_form=2)),
    (dict(kind=W.HEAT2D, nx=130, ny=257, nt=9), dict(m=4, k=3)),
    (dict(kind=W.HEAT2D, nx=16, ny=16, nt=64), dict(m=4, k=2, levels=3, m_coarse=2)),
    (dict(kind=W.HEAT2D, nx=16, ny=16, nt=64), dict(m=4, k=2, levels=3, m_coarse=2, nested=1)),
    (dict(kind=W.HEAT2D, nx=16, ny=16, nt=64), dict(m=4, k=2, levels=3, m_coarse=2, coarse_solver=2)),
    (dict(kind=W.HEAT2D, nx=0, ny=16, nt=32), dict(m=4, k=2)),            # refused: empty grid
    (dict(kind=W.HEAT2D, nx=16, ny=16, nt=32), dict(m=1, k=2)),           # refused: m < 2
    (dict(kind=W.HEAT2D, nx=16, ny=16, nt=3), dict(m=4, k=2)),            # refused: fewer steps than m
    (dict(kind=W.AC2D, nx=256, ny=256, nt=64), dict(m=4, k=2, coarse_solver=2, coarse_substeps=4)),
    (dict(kind=W.AC2D, nx=320, ny=256, nt=64), dict(m=4, k=2, coarse_solver=2)),  # refused: BF16 Psi, 320 columns
    (dict(kind=W.HEAT1D, nx=64, nt=64), dict(m=4, k=2, precision=1)),     # refused: FP32 form in 1D
    (dict(kind=9, nx=16, ny=16, nt=32), dict(m=4, k=2)),                  # refused: unknown kind
]

FIELDS = ("relax", "precision", "coarse_solver", "coarse_form", "levels", "m_coarse", "nested", "coarse_substeps")


def config_line(pd, od):
    o = W.Options(**od)
    p = W.Problem(**{"ny": 1, **pd})
    return p, o, " ".join(str(v) for v in (p.kind, p.nx, p.ny, p.nt, o.m, o.k, *(getattr(o, f) for f in FIELDS)))


@pytest.mark.skipif(shutil.which("hipcc") is None or shutil.which("gcc") is None, reason="needs hipcc and gcc")
def test_host_library_under_sanitizers():
    clangxx = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clangxx):
        pytest.skip("needs the ROCm clang++")
    with tempfile.TemporaryDirectory() as d:
        procs, objs = [], []
        for src in sorted(f for f in os.listdir(CSRC) if f.endswith(".hip")):
            obj = os.path.join(d, src[:-4] + ".o")
            cmd = ["hipcc", "-x", "hip", "--cuda-host-only", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17",
                   "-fPIC", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-c", os.path.join(CSRC, src), "-o", obj]
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
            objs.append(obj)
        for cmd, p in procs:
            _, err = p.communicate(timeout=600)
            assert p.returncode == 0, " ".join(cmd) + "\n" + err
        drv = os.path.join(d, "host_check.o")
        c = run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", *SAN, "-c",
                 os.path.join(HERE, "sanitize", "host_check.c"), "-o", drv])
        assert c.returncode == 0, c.stderr
        # the device code objects the host-only objects refer to, as empty stand-ins
        syms = set()
        for o in objs:
            nm = run(["nm", "-u", o])
            syms |= {line.split()[-1] for line in nm.stdout.splitlines() if "__hip_fatbin_" in line}
        stub = os.path.join(d, "fatbin_stub.c")
        with open(stub, "w") as f:
            for s in sorted(syms):
                f.write(f"char {s}[4096] __attribute__((aligned(4096)));\n")
        c = run(["gcc", "-c", stub, "-o", stub + ".o"])
        assert c.returncode == 0, c.stderr
        exe = os.path.join(d, "host_check")
        c = run([clangxx, "-fsanitize=address,undefined", drv, *objs, stub + ".o", "-L/opt/rocm/lib", "-lamdhip64",
                 "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
        assert c.returncode == 0, c.stderr
        lines = [config_line(pd, od) for pd, od in CONFIGS]
        r = subprocess.run([exe], input="\n".join(l for _, _, l in lines) + "\n", capture_output=True, text=True,
                           timeout=300, env=ENV)
        out = r.stdout + r.stderr
        assert r.returncode == 0 and "all checks passed" in r.stdout, out
        assert "runtime error" not in out and "AddressSanitizer" not in out, out
        rows = [tuple(int(v) for v in l.split()) for l in r.stdout.splitlines()[:len(lines)]]
        assert len(rows) == len(CONFIGS)
    # refused configurations have no workspace; the others agree with the production library
    import paper_2107_09596_amd as atm
    for (p, o, line), (ws, nt_intervals, status) in zip(lines, rows):
        assert ws == atm.atm_workspace_bytes(p, o), line
        if ws:
            assert status == atm.ATM_ERR_WORKSPACE and nt_intervals == atm.atm_num_intervals(p, o), line
        else:
            assert status != atm.ATM_OK, line
    assert sum(1 for _, (ws, _, _) in zip(lines, rows) if ws == 0) == 6
