"""Host-side logic of the driver that needs no GPU: the DIRK tableau the
stepper uses (section 2.3: Alexander's three-stage, third-order, L-stable
method), the argument checks that run before any device work, the mesh
descriptor marshalling, and the one-GPU bench's refusal of several GPUs."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_dirk_tableau():
    from paper_2608_27863_amd import pipeline
    A, b, d, e = pipeline.alexander_dirk()
    A, b, d, e = map(np.asarray, (A, b, d, e))
    g = A[0, 0]
    # gamma: the root of x^3 - 3x^2 + 3x/2 - 1/6 in (1/6, 1/2) that makes the method L-stable
    assert abs(g ** 3 - 3 * g ** 2 + 1.5 * g - 1.0 / 6.0) < 1e-15 and 1.0 / 6.0 < g < 0.5
    assert abs(g - 0.43586652150845899) < 1e-15
    assert np.allclose(np.diag(A), g) and np.all(np.triu(A, 1) == 0.0)
    assert np.array_equal(A[2], b)                       # stiffly accurate
    assert abs(A[1, 0] - (1 - g) / 2) < 1e-16
    c = A.sum(axis=1)
    # order conditions up to order 3
    assert abs(b.sum() - 1) < 1e-14
    assert abs(b @ c - 0.5) < 1e-14
    assert abs(b @ c ** 2 - 1.0 / 3.0) < 1e-14
    assert abs(b @ A @ c - 1.0 / 6.0) < 1e-14
    # d = A^{-1}, e = b^T d = (0, 0, 1) for a stiffly accurate tableau
    assert np.allclose(A @ d, np.eye(3), atol=1e-14)
    assert np.allclose(e, [0.0, 0.0, 1.0], atol=1e-14)
    # L-stability: R(z) = 1 + z b^T (I - z A)^{-1} 1 -> 0 as z -> -inf
    z = -1e8
    R = 1 + z * b @ np.linalg.solve(np.eye(3) - z * A, np.ones(3))
    assert abs(R) < 1e-6


def test_streamed_systems_need_the_mixed_path():
    from paper_2608_27863_amd import hdg, pipeline, synth
    wl = synth.config(0)
    for prec in (hdg.HDG_FP64, hdg.HDG_MIXED_FAST):
        with pytest.raises(ValueError, match="HDG_MIXED"):
            pipeline.NewtonStep(wl, prec=prec, stream_E=True)  # rejected before any device work


def test_descriptor_marshalling():
    from paper_2608_27863_amd import hdg, synth
    mesh = synth.curve_mesh(synth.box_mesh((3, 2, 2), p=2), 0.1)
    wl = synth.make_state(mesh, lambda x: synth.tgv_state(x, 0.5), mach=0.5, seed=1)
    desc, phys, keep = hdg.descriptors(mesh, wl)
    assert (desc.n_elem, desc.n_face, desc.n_vert) == (mesh.n_elem, mesh.n_face, mesh.n_vert)
    assert keep["ev"].dtype == np.int32 and np.array_equal(keep["ev"], mesh.elem_vert)
    assert keep["bc"].dtype == np.int8 and keep["p"].dtype == np.int8
    assert keep["geom"].shape == (mesh.n_elem, 27, 3) and desc.elem_geom == keep["geom"].ctypes.data
    assert (phys.gamma, phys.reynolds, phys.mach, phys.dt) == (wl.gamma, wl.reynolds, wl.mach, wl.dt)
    flat = synth.box_mesh((2, 2, 2), p=1)
    desc, _, keep = hdg.descriptors(flat, synth.make_state(flat, lambda x: synth.tgv_state(x, 0.5), mach=0.5))
    assert not desc.elem_geom and "geom" not in keep


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
