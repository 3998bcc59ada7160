"""Host-side checks of the C ABI: the built library exports every symbol the
header declares, the Python binding carries the same names, and descriptor
validation returns the documented codes before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hjpd.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(hjpd_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1803_01215_amd import hjpd
    return hjpd.load()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["hjpd_create", "hjpd_solve_batch", "hjpd_value_grad", "hjpd_destroy", "hjpd_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in _declared():
        assert hasattr(lib, n), n


def test_binding_has_same_names():
    from paper_1803_01215_amd import hjpd
    for n in _declared():
        assert callable(getattr(hjpd, n)), n
    assert sorted(hjpd.EXPORTED) == _declared()


def _desc(**kw):
    from paper_1803_01215_amd import hjpd
    base = dict(d=10, d_y=0, H=hjpd.HJPD_H_CNORM, g=hjpd.HJPD_G_QUAD_SHIFT, dtype=hjpd.HJPD_F32, N_max=32,
                sigma=1.0, tau=0.25, theta=1.0, tol=1e-6, max_iter=100, seed=1, flags=0, lanes_per_point=0,
                nodes_per_lane=0)
    base.update(kw)
    return hjpd.hjpd_desc(**base)


@pytest.mark.parametrize("bad", [
    dict(sigma=0.0), dict(sigma=-1.0), dict(tau=0.0), dict(sigma=1.0, tau=0.3), dict(theta=1.5), dict(theta=-0.1),
    dict(tol=0.0), dict(max_iter=0), dict(d=0), dict(N_max=0), dict(d_y=-1), dict(d_y=10), dict(dtype=7),
    dict(H=9), dict(g=9), dict(H=5), dict(g=5), dict(flags=1 << 10), dict(lanes_per_point=12, nodes_per_lane=1),
    dict(lanes_per_point=32, nodes_per_lane=5), dict(nodes_per_lane=2),
    dict(flags=64 | 128),                                # forward Euler and trapezoid together
])
def test_create_rejects_invalid_descriptors(lib, bad):
    from paper_1803_01215_amd import hjpd
    ctx = ctypes.c_void_p()
    rc = lib.hjpd_create(ctypes.byref(_desc(**bad)), ctypes.byref(ctx))
    assert rc == hjpd.HJPD_EINVAL
    assert ctx.value is None
    assert lib.hjpd_last_error().decode() != ""


@pytest.mark.parametrize("unsup", [
    dict(d=7),                                           # CNORM built for d in {2,3,4,10}
    dict(g=2),                                           # PAIR_DIST with the control path
    dict(H=1, d=10),                                     # quadrotor needs d = 12
    dict(H=2, d=12, d_y=0, g=2),                         # pursuit needs d_y = 6
    dict(H=3, d=100, g=3, dtype=1),                      # linear-tanh float32 only
    dict(N_max=300),                                     # beyond the largest tile
    dict(H=1, d=12, flags=32 | 1),                       # quadrotor Hopf: persistent kernel only
    dict(H=1, d=12, g=0, flags=32),                      # quadrotor Hopf: QUAD_SHIFT g only
    dict(H=2, d=12, d_y=6, g=2, flags=32),               # no Hopf for the game path
    dict(H=1, d=12, g=0, flags=64),                      # forward Euler: quadrotor with QUAD_SHIFT g only
    dict(H=2, d=12, d_y=6, g=2, flags=128),              # no trapezoid for the game path
    dict(flags=64 | 1),                                  # no weighted discretisation on the plain kernel
    dict(flags=128 | 32),                                # nor with the Hopf formulation
    dict(flags=64, starts=3),                            # nor with the recipes
    dict(H=2, d=12, d_y=6, g=2, starts=2),               # one start on the game path
    dict(H=4, g=4, d=2, d_y=1, restarts=1),              # no recipes for Isaacs' game
    dict(H=2, d=12, d_y=6, g=2, restarts=1, flags=1),    # nor on the plain kernel
    dict(H=4, g=4, d=2, d_y=1, flags=32 | 1),            # Isaacs: no plain kernel, Algorithm 4
    dict(H=4, g=4, d=2, d_y=1, flags=1),                 # nor Algorithm 3
    dict(H=4, g=4, d=3, d_y=1, flags=32),                # scalar players only
    dict(H=4, g=1, d=2, d_y=1, flags=32),                # Isaacs pairs with SADDLE_QUAD
    dict(g=4, d=10, flags=32),                           # SADDLE_QUAD is a game cost
])
def test_create_reports_unsupported(lib, unsup):
    from paper_1803_01215_amd import hjpd
    ctx = ctypes.c_void_p()
    assert lib.hjpd_create(ctypes.byref(_desc(**unsup)), ctypes.byref(ctx)) == hjpd.HJPD_EUNSUPPORTED


def test_null_arguments(lib):
    from paper_1803_01215_amd import hjpd
    assert lib.hjpd_create(None, None) == hjpd.HJPD_EINVAL
    assert lib.hjpd_solve_batch(None, 1, None, None, None, None, None, None, None, None, None, None, None) == \
        hjpd.HJPD_EINVAL
    assert lib.hjpd_destroy(None) == hjpd.HJPD_OK
    ms = ctypes.c_double()
    assert lib.hjpd_get_timing(None, ctypes.byref(ms), None) == hjpd.HJPD_EINVAL


@pytest.mark.parametrize("ok", [dict(), dict(H=4, g=4, d=2, d_y=1), dict(H=4, g=4, d=2, d_y=1, flags=32),
                                dict(H=2, d=12, d_y=6, g=2, restarts=2, sigma_inc=20.0, value_tol=1e-9),
                                dict(H=1, d=12, flags=64), dict(H=1, d=12, flags=128, N_max=200)])
def test_valid_descriptor_without_gpu_reports_device_error(lib, ok):
    """Descriptors that validate (eikonal; Isaacs' game by Algorithm 3 and by
    Algorithm 4; the pursuit-evasion game with the sigma and value-change
    recipes; forward Euler and trapezoid for the quadrotor) get as far as the
    device query."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1803_01215_amd import hjpd
    ctx = ctypes.c_void_p()
    assert lib.hjpd_create(ctypes.byref(_desc(**ok)), ctypes.byref(ctx)) == hjpd.HJPD_EDEVICE


def test_flag_values_match_header():
    """The binding's flag constants are the header's (shift expressions parsed)."""
    from paper_1803_01215_amd import hjpd
    src = open(HEADER).read()
    for name in ["HJPD_PLAIN", "HJPD_FIXED_ITERS", "HJPD_GRAPH", "HJPD_TIMING", "HJPD_NO_ORDER_HINT", "HJPD_HOPF",
                 "HJPD_FORWARD_EULER", "HJPD_TRAPEZOID"]:
        m = re.search(name + r"\s*=\s*1u\s*<<\s*(\d+)", src)
        assert m, name
        assert getattr(hjpd, name) == 1 << int(m.group(1)), name


def test_library_shares_torchs_hip_runtime():
    """Loading the library through the binding, before anything imported
    torch, leaves one HIP runtime in the process: torch's copy."""
    import subprocess
    import sys
    code = ("import re\n"
            "from paper_1803_01215_amd import hjpd\n"
            "hjpd.load()\n"
            "print(sorted(set(re.findall(r'\\S*libamdhip64\\S*', open('/proc/self/maps').read()))))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, check=True).stdout
    libs = eval(out.strip())
    assert len(libs) == 1 and "/torch/lib/" in libs[0], libs


@pytest.mark.parametrize("args", [(2, 8, 1, 10), (0, 3, 1, 10), (0, 8, 0, 10), (0, 8, 9, 10), (1, 8, 1, 0)])
def test_calibrate_fma_rejects_bad_arguments(lib, args):
    """Bad dtype, chain count, waves per SIMD or rounds: EINVAL before any device call."""
    from paper_1803_01215_amd import hjpd
    ms = ctypes.c_double()
    assert lib.hjpd_calibrate_fma(*args[:3], ctypes.c_int64(args[3]), ctypes.byref(ms), None, None) == hjpd.HJPD_EINVAL
    assert lib.hjpd_calibrate_fma(0, 8, 1, ctypes.c_int64(10), None, None, None) == hjpd.HJPD_EINVAL
