"""Host-side checks of the HIP library that need no GPU: it loads, exports
every function include/gplbm.h declares, and validates parameters."""
import ctypes
import os
import re

import pytest

import workloads as wl
from paper_2111_05960_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    with open(os.path.join(ROOT, "include", "gplbm.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gplbm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2111_05960_amd import build
    if build.stale():
        build.build()
    return B.load()


def test_every_declared_function_is_exported(lib):
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.SYMBOLS)


def test_struct_sizes_match_header(lib):
    assert ctypes.sizeof(B.gplbm_params) == 4 * 14 + 8 * 16
    assert ctypes.sizeof(B.gplbm_diag) == 8 * 7 + 8


def test_state_bytes_layout(lib):
    p = wl.base_params(lattice=wl.D3Q19, shape=(16, 12, 10), bc=(0, 0, 0))
    for prec, elem in (("fp64", 8), ("fp32", 4)):
        cp = B.make_params(p, prec)
        n = 16 * 12 * 10
        rnd = lambda v: (v + 255) // 256 * 256
        pop, phi = rnd(19 * n * elem), rnd(n * elem)
        assert B.gplbm_checkpoint_bytes(cp) == 2 * pop + phi
        assert B.gplbm_state_bytes(cp) >= 4 * pop + 2 * phi


@pytest.mark.parametrize("prec", ["fp16dev", "bf16dev"])
@pytest.mark.parametrize("lattice,shape,q,hl,qh", [
    (wl.D3Q19, (16, 12, 10), 19, 0, 19), (wl.D2Q9, (1, 12, 10), 9, 0, 9),
    (wl.D3Q19, (16, 12, 10), 19, 1, 7), (wl.D2Q9, (1, 12, 10), 9, 1, 5)])
def test_state_bytes_layout_deviation(lib, prec, lattice, shape, q, hl, qh):
    """Deviation formats: each distribution is its lattice's Q - 1 16-bit
    moving populations and an FP32 rest population per node (h on the light
    lattice: Qh - 1 of them); phi and Lambda FP32."""
    n = shape[0] * shape[1] * shape[2]
    rnd = lambda v: (v + 255) // 256 * 256
    cp = B.make_params(wl.base_params(lattice=lattice, shape=shape, bc=(0, 0, 0), h_lattice=hl),
                       prec)
    dist_g = rnd((q - 1) * n * 2) + rnd(n * 4)
    dist_h = rnd((qh - 1) * n * 2) + rnd(n * 4)
    assert B.gplbm_checkpoint_bytes(cp) == dist_g + dist_h + 2 * rnd(n * 4)
    assert B.gplbm_state_bytes(cp) >= 2 * (dist_g + dist_h) + 4 * rnd(n * 4)


@pytest.mark.parametrize("prec", ["fp16dev", "bf16dev"])
def test_deviation_storage_accepted_on_every_lattice(lib, prec):
    for lattice, shape in ((wl.D2Q9, (1, 64, 64)), (wl.D3Q19, (8, 8, 8)), (wl.D2Q5, (1, 64, 64)),
                           (wl.D3Q7, (8, 8, 8))):
        p = wl.base_params(lattice=lattice, shape=shape, bc=(0, 0, 0))
        assert B.gplbm_state_bytes(B.make_params(p, prec)) > 0


@pytest.mark.parametrize("lattice,shape,qg,qh", [
    (wl.D3Q19, (16, 12, 10), 19, 7), (wl.D2Q9, (1, 12, 10), 9, 5)])
def test_state_bytes_layout_light_h(lib, lattice, shape, qg, qh):
    """h on D2Q5 / D3Q7: the h distribution holds Qh populations per node."""
    p = wl.base_params(lattice=lattice, shape=shape, bc=(0, 0, 0), h_lattice=1)
    n = shape[0] * shape[1] * shape[2]
    rnd = lambda v: (v + 255) // 256 * 256
    for prec, elem in (("fp64", 8), ("fp32", 4)):
        cp = B.make_params(p, prec)
        assert cp.h_lattice == 1
        pg, ph, phi = rnd(qg * n * elem), rnd(qh * n * elem), rnd(n * elem)
        assert B.gplbm_checkpoint_bytes(cp) == pg + ph + phi
        assert B.gplbm_state_bytes(cp) >= 2 * pg + 2 * ph + 2 * phi
        full = B.make_params(dict(p, h_lattice=0), prec)
        assert B.gplbm_state_bytes(full) - B.gplbm_state_bytes(cp) == 2 * (pg - ph)


def test_adjoint_workspace_light_h(lib):
    """With h on D3Q7 the adjoint of the h populations (B1) holds 7 values
    per node, the adjoint of the g populations (A1) 19."""
    shape = (8, 8, 8)
    n = 8 * 8 * 8
    rnd = lambda v: (v + 255) // 256 * 256
    out = ctypes.c_uint64()
    full = B.make_params(wl.base_params(lattice=wl.D3Q19, shape=shape, bc=(0, 0, 0)), "fp64")
    light = B.make_params(wl.base_params(lattice=wl.D3Q19, shape=shape, bc=(0, 0, 0),
                                         h_lattice=1), "fp64")
    assert lib.gplbm_adjoint_bytes(ctypes.byref(full), ctypes.byref(out)) == B.GPLBM_OK
    bf = out.value
    assert lib.gplbm_adjoint_bytes(ctypes.byref(light), ctypes.byref(out)) == B.GPLBM_OK
    assert bf - out.value == 2 * (rnd(19 * n * 8) - rnd(7 * n * 8))


@pytest.mark.parametrize("field,value", [
    ("M_phi", 0.0), ("M_phi", -1.0), ("gamma", 0.0), ("W", 0.0), ("nz", 2), ("nx", 0),
    ("lattice", 7), ("lattice", 4), ("precision", 9), ("schedule", 5), ("lam", float("nan")),
    ("h_lattice", 2), ("h_lattice", -1),
])
def test_invalid_parameters_rejected(lib, field, value):
    p = wl.base_params()
    cp = B.make_params(p)
    setattr(cp, field, value)
    with pytest.raises(B.GplbmError) as e:
        B.gplbm_state_bytes(cp)
    assert e.value.code == B.GPLBM_E_INVALID
    # gplbm_create rejects the same parameters before touching the device
    h = ctypes.c_void_p()
    rc = lib.gplbm_create(ctypes.byref(cp), ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(h))
    assert rc == B.GPLBM_E_INVALID and not h.value


def test_create_rejects_small_or_misaligned_buffer(lib):
    cp = B.make_params(wl.base_params())
    need = B.gplbm_state_bytes(cp)
    h = ctypes.c_void_p()
    assert lib.gplbm_create(ctypes.byref(cp), ctypes.c_void_p(4096), need - 1, None,
                            ctypes.byref(h)) == B.GPLBM_E_SIZE
    assert lib.gplbm_create(ctypes.byref(cp), ctypes.c_void_p(4096 + 8), need, None,
                            ctypes.byref(h)) == B.GPLBM_E_INVALID
    assert lib.gplbm_create(ctypes.byref(cp), None, need, None,
                            ctypes.byref(h)) == B.GPLBM_E_INVALID


def test_null_context_is_rejected(lib):
    assert lib.gplbm_step(None, 1) == B.GPLBM_E_INVALID
    assert lib.gplbm_init_fields(None, None, None) == B.GPLBM_E_INVALID
    assert lib.gplbm_step_count(None) == -1
    assert lib.gplbm_step_chain(None, None, 256, 1) == B.GPLBM_E_INVALID
    assert lib.gplbm_adjoint_segment(None, None, 256, 1) == B.GPLBM_E_INVALID


@pytest.mark.parametrize("prec", ["fp16dev", "bf16dev"])
@pytest.mark.parametrize("over", [dict(h_scheme=1), dict(free_energy=1, eps_s=1.0, eps_l=2.0)])
def test_variants_accepted_with_deviation_storage(lib, prec, over):
    """h^eq,alt and general free energies change no array of the deviation
    formats: same state size as the base scheme."""
    base = wl.base_params(lattice=wl.D3Q19, shape=(8, 8, 8), bc=(0, 0, 0))
    assert (B.gplbm_state_bytes(B.make_params(dict(base, **over), prec))
            == B.gplbm_state_bytes(B.make_params(base, prec)))


@pytest.mark.parametrize("over", [dict(h_scheme=1), dict(free_energy=1, eps_s=1.0, eps_l=2.0)])
def test_adjoint_workspace_variants(lib, over):
    """The scheme variants change no array of the adjoint: same workspace as
    the base scheme."""
    base = B.make_params(wl.base_params(lattice=wl.D2Q9, shape=(1, 8, 8), bc=(0, 0, 0)), "fp64")
    cp = B.make_params(wl.base_params(lattice=wl.D2Q9, shape=(1, 8, 8), bc=(0, 0, 0), **over),
                       "fp64")
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    assert lib.gplbm_adjoint_bytes(ctypes.byref(base), ctypes.byref(a)) == B.GPLBM_OK
    assert lib.gplbm_adjoint_bytes(ctypes.byref(cp), ctypes.byref(b)) == B.GPLBM_OK
    assert a.value == b.value > 0


@pytest.mark.parametrize("prec", ["fp16dev", "bf16dev"])
def test_adjoint_workspace_deviation_storage(lib, prec):
    """The reverse sweep is FP64 whatever the forward storage: a deviation
    context needs the FP64 context's workspace."""
    p = wl.base_params(lattice=wl.D3Q19, shape=(8, 8, 8), bc=(0, 0, 0))
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    assert lib.gplbm_adjoint_bytes(ctypes.byref(B.make_params(p, "fp64")), ctypes.byref(a)) == B.GPLBM_OK
    assert lib.gplbm_adjoint_bytes(ctypes.byref(B.make_params(p, prec)), ctypes.byref(b)) == B.GPLBM_OK
    assert a.value == b.value > 0


def test_adjoint_bytes_rejects_invalid_parameters(lib):
    out = ctypes.c_uint64()
    p = wl.base_params(lattice=wl.D3Q19, shape=(8, 8, 8), bc=(0, 0, 0), h_lattice=1)
    assert lib.gplbm_adjoint_bytes(ctypes.byref(B.make_params(p, "fp16dev")),
                                   ctypes.byref(out)) == B.GPLBM_OK
    cp = B.make_params(p, "fp16dev")
    cp.nz = 0
    assert lib.gplbm_adjoint_bytes(ctypes.byref(cp), ctypes.byref(out)) == B.GPLBM_E_INVALID


@pytest.mark.parametrize("field,value", [("h_scheme", 2), ("free_energy", 3), ("eps_s", 0.0),
                                         ("eps_l", -1.0), ("m_s", float("inf"))])
def test_variant_parameters_validated(lib, field, value):
    cp = B.make_params(wl.base_params(free_energy=1, eps_s=1.0, eps_l=2.0))
    assert B.gplbm_state_bytes(cp) > 0
    setattr(cp, field, value)
    with pytest.raises(B.GplbmError) as e:
        B.gplbm_state_bytes(cp)
    assert e.value.code == B.GPLBM_E_INVALID


@pytest.mark.parametrize("lattice,shape,q", [(wl.D2Q5, (1, 12, 10), 5), (wl.D3Q7, (6, 12, 10), 7)])
def test_state_bytes_layout_light_g(lib, lattice, shape, q):
    """g on D2Q5 / D3Q7: both distributions hold Q populations of that lattice."""
    p = wl.base_params(lattice=lattice, shape=shape, bc=(0, 0, 0))
    n = shape[0] * shape[1] * shape[2]
    rnd = lambda v: (v + 255) // 256 * 256
    cp = B.make_params(p, "fp64")
    assert B.gplbm_checkpoint_bytes(cp) == 2 * rnd(q * n * 8) + rnd(n * 8)
    out = ctypes.c_uint64()
    assert lib.gplbm_adjoint_bytes(ctypes.byref(cp), ctypes.byref(out)) == B.GPLBM_OK
    for prec in ("fp16dev", "bf16dev"):
        # deviation formats: Q - 1 16-bit codes and an FP32 rest population
        dist = rnd((q - 1) * n * 2) + rnd(n * 4)
        assert B.gplbm_checkpoint_bytes(B.make_params(p, prec)) == 2 * dist + 2 * rnd(n * 4)
    bad = B.make_params(dict(p, shape=(2,) + shape[1:]) if lattice == wl.D2Q5 else p, "fp64")
    if lattice == wl.D2Q5:
        with pytest.raises(B.GplbmError):
            B.gplbm_state_bytes(bad)


def test_unit_conversion_matches_the_paper_runs():
    """The physical parameters of the Sec. 4.2 dissolution run (M_phi = 1.2,
    D_l = 1, D_s = 0, W = 5e-3, dx = 1e-4, dt = 5e-9) convert to the lattice
    parameters the validation workload states directly (M, D x 0.5, W = 50
    cells), and t = 5e-4 is 1e5 steps."""
    from paper_2111_05960_amd import units
    p, _, _ = wl.paper_validation("dissolution")
    phys = dict(p, M_phi=1.2, D_l=1.0, D_s=0.0, W=5e-3)
    del phys["gamma"]
    lat = units.to_lattice_units(phys, wl.PAPER_DX, wl.PAPER_DT)
    for k in ("M_phi", "D_l", "D_s", "W", "gamma", "lam", "c_s_co", "c_l_co", "mu_eq"):
        assert abs(lat[k] - p[k]) <= 1e-12 * max(abs(p[k]), 1.0), k
    assert units.lattice_steps(5e-4, wl.PAPER_DT) == 100000
    with pytest.raises(ValueError):
        units.lattice_steps(5e-4 + 1e-9, wl.PAPER_DT)
    back = units.to_lattice_units(dict(gamma=2.0), 0.5, 0.25)
    assert back["gamma"] == 2.0 / (0.25 / 0.25)


def test_missing_library_fails_loudly(tmp_path):
    """With the library absent the binding raises instead of falling back to
    any other implementation (there is none)."""
    import subprocess
    import sys
    code = (
        "from paper_2111_05960_amd import binding\n"
        "try:\n"
        "    binding.load()\n"
        "except RuntimeError as e:\n"
        "    assert 'missing' in str(e) and 'no fallback' in str(e), e\n"
        "    print('raised')\n"
    )
    env = dict(os.environ, GPLBM_LIBRARY=str(tmp_path / "absent.so"))
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "raised"
