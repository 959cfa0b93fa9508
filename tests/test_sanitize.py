"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle's C (gcc, sanitized) computes element systems, condensations and
  LU factors on meshes with every boundary type (p = 1, 2) and on a curved
  mesh.
* The library's host pass (hipcc with the sanitizers on the host side only;
  the device code is unchanged) runs hdg_create's whole set-up -- validation,
  geometry (straight and curved), face numbering, the block-sparse pattern,
  gather lists, vertex classes -- on five meshes up to 2000 mixed-degree
  elements; without a GPU the first HIP call then fails and hdg_create returns
  HDG_ERR_DEVICE through its cleanup path.  A descriptor with a vertex index
  out of range is rejected before any of it.
* A positive control: a planted heap overflow in a throwaway C file is
  reported by the same harness, so a harness that fails to detect would fail
  this test.

Each case runs in a child Python process with the sanitizer runtime preloaded.
Leak checking is off (the interpreter itself does not free everything)."""
import glob
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


def _gcc_runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _child(code, preload, args, timeout=600):
    env = dict(os.environ, LD_PRELOAD=preload, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONPATH=ROOT)
    return subprocess.run([sys.executable, "-c", textwrap.dedent(code), *args], env=env, capture_output=True,
                          text=True, timeout=timeout)


ORACLE_CHILD = """
    import sys
    from oracle import oracle as O
    O._LIB = sys.argv[1]
    from paper_2608_27863_amd import synth
    types = {(0, 0): 1, (0, 1): 2, (1, 0): 3, (1, 1): 4, (2, 0): 5, (2, 1): 5}
    f = lambda x: synth.tgv_state(x, 0.8)
    for p in (1, 2):
        m = synth.set_boundary_types(synth.box_mesh((2, 2, 2), lengths=(2.0, 1.5, 1.0), periodic=(False,) * 3,
                                                    p=p, perturb=0.1, seed=4), types)
        wl = synth.make_state(m, f, mach=0.8, noise=1e-2, nu_amp=3e-4, seed=4, reynolds=80.0, boundary_field=f)
        sz = O.Sizes(m)
        for e in (0, 7):
            E = O.element_system(wl, e, sz)
            O.condense(E, sz.n(e))
            O.LU(E[:sz.n(e), :sz.n(e)])
    cm = synth.curve_mesh(synth.box_mesh((2, 2, 2), p=2), 0.2)
    wl = synth.make_state(cm, lambda x: synth.tgv_state(x, 1.25), mach=1.25, noise=1e-3, seed=3)
    O.element_system(wl, 3)
    O.element_volume(cm, 3)
    print("oracle done")
"""

HOST_CHILD = """
    import ctypes, sys
    from paper_2608_27863_amd import hdg, synth
    L = hdg.load_library(sys.argv[1])
    types = {(0, 0): 1, (0, 1): 2, (1, 0): 3, (1, 1): 4, (2, 0): 5, (2, 1): 5}
    f = lambda x: synth.tgv_state(x, 0.8)
    meshes = [synth.set_boundary_types(synth.box_mesh((2, 2, 2), lengths=(2.0, 1.5, 1.0), periodic=(False,) * 3,
                                                      p=p, perturb=0.1, seed=4), types) for p in (1, 2, 4)]
    meshes.append(synth.curve_mesh(synth.box_mesh((2, 2, 2), p=3), 0.2))
    meshes.append(synth.config(3).mesh)
    for m in meshes:
        wl = synth.make_state(m, f, mach=0.8, noise=0.0, seed=1, boundary_field=f)
        desc, phys, keep = hdg.descriptors(m, wl)
        h = hdg._vp()
        rc = L.hdg_create(ctypes.byref(desc), ctypes.byref(phys), ctypes.byref(h))
        assert rc == -4 and not h.value, rc  # HDG_ERR_DEVICE: no GPU here, after the whole host set-up
        desc, phys, keep = hdg.descriptors(m, wl)
        keep["ev"][m.n_elem // 2, 3] = m.n_vert
        assert L.hdg_create(ctypes.byref(desc), ctypes.byref(phys), ctypes.byref(h)) == -1
    print("host done")
"""

CONTROL_C = """
    #include <stdlib.h>
    int planted_overflow(int n) {
        int *a = (int *)malloc(sizeof(int) * n);
        for (int i = 0; i <= n; ++i) a[i] = i;  /* one element past the end */
        int s = a[0];
        free(a);
        return s;
    }
"""

CONTROL_CHILD = """
    import ctypes, sys
    ctypes.CDLL(sys.argv[1]).planted_overflow(8)
    print("control done")
"""


@pytest.fixture(scope="module")
def gcc_asan():
    rt = _gcc_runtime("libasan.so")
    if rt is None or shutil.which("gcc") is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    return rt


def test_harness_detects_a_planted_overflow(tmp_path, gcc_asan):
    src = tmp_path / "control.c"
    src.write_text(textwrap.dedent(CONTROL_C))
    lib = tmp_path / "libcontrol.so"
    subprocess.check_call(["gcc", "-O0", "-g", "-fsanitize=address,undefined", "-shared", "-fPIC",
                           "-o", str(lib), str(src)])
    r = _child(CONTROL_CHILD, gcc_asan, [str(lib)])
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr, r.stderr[-2000:]


def test_oracle_under_sanitizers(tmp_path, gcc_asan):
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-std=c99", "-D_DEFAULT_SOURCE", "-shared", "-fPIC", "-o", str(lib),
                           os.path.join(ROOT, "oracle", "hdgref.c"), "-lm"])
    r = _child(ORACLE_CHILD, gcc_asan, [str(lib)])
    print(r.stdout[-500:])
    assert r.returncode == 0 and "oracle done" in r.stdout, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]


def test_library_host_setup_under_sanitizers(tmp_path):
    rt = _clang_asan_runtime()
    if rt is None or not os.path.exists(HIPCC):
        pytest.skip("hipcc or clang's AddressSanitizer runtime is not installed")
    from paper_2608_27863_amd import build
    objdir = os.path.join(ROOT, "paper_2608_27863_amd", "_build")
    kernels = sorted(glob.glob(os.path.join(objdir, "k_*.hip.o")))
    if len(kernels) != len([s for s in build.sources() if os.path.basename(s).startswith("k_")]):
        build.build()
        kernels = sorted(glob.glob(os.path.join(objdir, "k_*.hip.o")))
    host_obj = tmp_path / "hdg_host_san.o"
    # the sanitizers apply to the host pass only (each flag right after -Xarch_host)
    subprocess.check_call([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={build.ARCH}",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-omit-frame-pointer",
                           "-x", "hip", "-c", os.path.join(ROOT, "paper_2608_27863_amd", "csrc", "hdg_host.cpp"),
                           "-o", str(host_obj)], stderr=subprocess.DEVNULL)
    lib = tmp_path / "libhdg_san.so"
    subprocess.check_call([HIPCC, "-shared", "-fPIC", f"--offload-arch={build.ARCH}", "-o", str(lib), str(host_obj),
                           *kernels, rt, f"-Wl,-rpath,{os.path.dirname(rt)}"])
    r = _child(HOST_CHILD, rt, [str(lib)])
    print(r.stdout[-500:])
    assert r.returncode == 0 and "host done" in r.stdout, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
