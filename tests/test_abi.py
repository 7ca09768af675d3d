"""CPU checks of the C ABI: the library loads, exports every declared symbol, and its host-only
helpers agree with the oracle (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hx.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hx_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["hx_setup", "hx_destroy", "hx_residual", "hx_update_linearization",
                     "hx_apply_tangent", "hx_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2408_12479_amd as hx
    lib = ctypes.CDLL(hx.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings():
    import paper_2408_12479_amd as hx
    for code in range(9):
        assert hx.lib.hx_status_string(code)
    assert hx.lib.hx_status_string(5).decode().startswith("inverted")


def test_fiber_structure_matches_oracle_and_table():
    import paper_2408_12479_amd as hx
    from oracle import fiber
    E = np.eye(3)
    phi = np.deg2rad(27.47)
    H4, H6, M4, M6 = hx.fiber_structure(3.62, 34.3, phi, E)
    h11, h22, h33 = fiber.dispersion_coefficients(3.62, 34.3)
    oH4, oH6, oM4, oM6 = fiber.structure_tensors(E[0], E[1], E[2], phi, h11, h22, h33)
    np.testing.assert_allclose(H4, oH4, atol=1e-15)
    np.testing.assert_allclose(H6, oH6, atol=1e-15)
    np.testing.assert_allclose(M4, oM4, atol=1e-15)
    np.testing.assert_allclose(M6, oM6, atol=1e-15)
    # table of fibre parameters: 0.9168, 0.0759, 0.0073 along M1, M2, M3 of family 4
    R = np.stack([M4, [-np.sin(phi), np.cos(phi), 0.0], [0, 0, 1.0]])
    np.testing.assert_allclose(np.diag(R @ H4 @ R.T), [0.9168, 0.0759, 0.0073], atol=5e-5)


def test_fiber_structure_rejects_bad_input():
    import paper_2408_12479_amd as hx
    with pytest.raises(hx.HxError):
        hx.fiber_structure(3.62, -1.0, 0.3)


def test_one_hip_runtime_per_process():
    """Importing the binding in a fresh process maps a single HIP runtime (torch's): libhx.so must
    not bring a second libamdhip64 next to the one torch loads."""
    import subprocess
    import sys
    code = ("import paper_2408_12479_amd, torch\n"
            "torch.cuda.is_available()\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_setup_refuses_empty_and_degenerate_meshes():
    """hx_setup_lattice and hx_setup check their arguments on the host before any device call: an
    empty lattice, a mesh without cells or with fewer than 8 vertices, a degree outside [1, 6] and
    NULL arguments all come back as errors with no context."""
    import paper_2408_12479_amd as hx
    for dims in ((0, 2, 2), (2, 0, 2), (2, 2, 0)):
        V = np.zeros((dims[2] + 1) * (dims[1] + 1) * (dims[0] + 1) * 3)
        with pytest.raises(hx.HxError) as err:
            hx.Operator(*dims, V, 2, law="cnh", mu=1.0, lam=1.0)
        assert err.value.name == "HX_E_ARG"
        assert "empty lattice" in str(err.value)
    V8 = np.array([[a, b, c] for c in (0.0, 1.0) for b in (0.0, 1.0) for a in (0.0, 1.0)])
    with pytest.raises(hx.HxError) as err:
        hx.HexOperator(V8, np.zeros((0, 8), dtype=np.int64), 2, law="cnh", mu=1.0, lam=1.0)
    assert err.value.name == "HX_E_ARG"
    assert "at least one cell" in str(err.value)
    with pytest.raises(hx.HxError) as err:
        hx.HexOperator(V8[:7], np.arange(8)[None] % 7, 2, law="cnh", mu=1.0, lam=1.0)
    assert err.value.name == "HX_E_ARG"
    for p in (0, 7):
        with pytest.raises(hx.HxError) as err:
            hx.HexOperator(V8, np.arange(8)[None], p, law="cnh", mu=1.0, lam=1.0)
        assert err.value.name == "HX_E_UNSUPPORTED"
    ctx = ctypes.c_void_p()
    assert hx.STATUS[hx.lib.hx_setup_lattice(None, 2, None, None, ctypes.byref(ctx))] == "HX_E_ARG"
    assert hx.STATUS[hx.lib.hx_setup(None, 2, None, None, ctypes.byref(ctx))] == "HX_E_ARG"
    assert ctx.value is None
    assert hx.STATUS[hx.lib.hx_setup(None, 2, None, None, None)] == "HX_E_ARG"
