"""Host-side sanitizer builds (CPU only): the C oracle built with AddressSanitizer
and UndefinedBehaviorSanitizer runs its operator, clover term, sampled apply
and link derivative without a report and with the results of the plain build;
the library's host code built with both sanitizers (device code untouched)
runs the entry points that need no device (version, argument checks, the
no-device error of create) without a report."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gcc_runtime(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()


ORACLE_SCRIPT = r"""
import sys
import numpy as np
sys.path.insert(0, {root!r})
import oracle
from paper_2407_00041_amd import synth
oracle._SO = {so!r}
oracle._lib = None
dims = (2, 4, 2, 6)
U = synth.smooth_links(dims, 3).numpy()
psi = synth.gaussian_spinor(dims, 4, nrhs=2)
out = {{}}
out["apply"] = oracle.dirac_apply(dims, U, psi, -0.3, 1.0, antiperiodic_t=True)
out["adjoint"] = oracle.dirac_apply(dims, U, psi, -0.3, 1.0, dagger=True)
out["clover"] = oracle.clover_term(dims, U)
sites = np.array([0, 5, 17, 40, 95])
out["sites"] = oracle.dirac_apply_sites(dims, U, psi[0], sites, -0.3, 1.0)
G, F = oracle.force_links(dims, U, psi[1], psi[0], sites, np.array([0, 1, 2, 3, 0]), csw=1.0)
out["force"] = F
np.savez({npz!r}, **out)
"""


def _run_oracle(so, npz, env_extra):
    env = dict(os.environ, **env_extra)
    code = ORACLE_SCRIPT.format(root=ROOT, so=so, npz=npz)
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300)


def test_oracle_under_asan_and_ubsan():
    import numpy as np
    src = os.path.join(ROOT, "oracle", "oracle.c")
    with tempfile.TemporaryDirectory() as d:
        san = os.path.join(d, "liboracle_san.so")
        plain = os.path.join(d, "liboracle_plain.so")
        subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-omit-frame-pointer",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-o", san, src, "-lm"])
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", plain, src, "-lm"])
        r = _run_oracle(san, os.path.join(d, "san.npz"),
                        {"LD_PRELOAD": _gcc_runtime("libasan.so") + ":" + _gcc_runtime("libubsan.so"),
                         "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1",
                         "OMP_NUM_THREADS": "2"})
        assert r.returncode == 0 and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, \
            r.stderr[-3000:]
        r2 = _run_oracle(plain, os.path.join(d, "plain.npz"), {"OMP_NUM_THREADS": "2"})
        assert r2.returncode == 0, r2.stderr[-2000:]
        a, b = np.load(os.path.join(d, "san.npz")), np.load(os.path.join(d, "plain.npz"))
        for k in a.files:
            assert np.allclose(a[k], b[k], rtol=1e-12, atol=1e-13), k


LIB_SCRIPT = r"""
import ctypes, sys
sys.path.insert(0, {root!r})
from paper_2407_00041_amd import _lib
_lib.SO_PATH = {so!r}
lib = _lib.load()
assert lib.dirac_version().startswith(b"wdirac")
assert lib.dirac_apply(None, None, None, 1, 0, None) == _lib.EINVAL
assert lib.dirac_force_workspace_bytes(None) == 0
assert lib.fgmres_workspace_bytes(None, None, 1) == 0
assert lib.dirac_amg_restrict(None, None, None, 1, None) == _lib.EINVAL
assert lib.dirac_amg_destroy(None) == 0
h = ctypes.c_void_p()
dims = (ctypes.c_int * 4)(4, 4, 4, 4)
links = (ctypes.c_double * (2 * 256 * 36))()
rc = lib.dirac_create(ctypes.byref(h), dims, links, None, -0.3, 1.0, 0)
assert rc < 0 and not h.value, rc      # no HIP device in this container
print("ok", lib.dirac_last_error().decode())
"""


def test_library_host_code_under_asan_and_ubsan():
    sys.path.insert(0, ROOT)
    from paper_2407_00041_amd import build as hipbuild
    rt = subprocess.run(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True).stdout.strip()
    if not os.path.exists(rt):
        pytest.skip("clang's ASan runtime is not installed")
    with tempfile.TemporaryDirectory() as d:
        so = os.path.join(d, "libwdirac_san.so")
        # sanitizers on the host side of every translation unit only (the device code is built as usual)
        flags = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
        # the shared object leaves the sanitizer runtime's symbols undefined: the preloaded runtime provides them
        hipbuild.build(out=so, build_dir=os.path.join(d, "objs"), extra=flags)
        env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1")
        r = subprocess.run([sys.executable, "-c", LIB_SCRIPT.format(root=ROOT, so=so)], capture_output=True,
                           text=True, env=env, timeout=300)
        assert r.returncode == 0 and r.stdout.startswith("ok"), (r.stdout[-2000:], r.stderr[-3000:])
        assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
