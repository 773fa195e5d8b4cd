"""The C interface: the library loads without a GPU and exports every function that
include/fdlb.h declares; host-only calls (sizes, validation, strings) behave as documented.
No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdlb.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdlb_[a-z_]+)\s*\(", text)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ("fdlb_create", "fdlb_set_state", "fdlb_step", "fdlb_get_moments", "fdlb_destroy",
              "fdlb_batch_create", "fdlb_batch_set_state", "fdlb_batch_get_moments", "fdlb_get_f", "fdlb_set_f",
              "fdlb_diag", "fdlb_required_bytes", "fdlb_batch_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_0801_4169_amd import _binding as B
    lib = ctypes.CDLL(B.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
        assert n in B.EXPORTED, f"binding lacks {n}"


def _sod_params(**kw):
    import fdlb_inputs as fi
    from paper_0801_4169_amd import _binding as B
    p, _, _ = fi.sod_tube()
    prm = B.make_params(p)
    for k, v in kw.items():
        setattr(prm, k, v)
    return prm


def test_required_bytes_layout():
    from paper_0801_4169_amd import _binding as B
    prm = _sod_params()
    n64 = B.fdlb_required_bytes(prm)
    prm32 = _sod_params(precision=B.FDLB_F32)
    n32 = B.fdlb_required_bytes(prm32)
    # two halves of 33 planes (pitch rounded to 32 cells) plus pressure rows
    assert n64 >= 2 * 33 * 4 * 416 * 8 and n32 >= 2 * 33 * 4 * 416 * 4 and n32 < n64


@pytest.mark.parametrize("field,value", [("nx", 0), ("dt", 0.0), ("tau", -1.0), ("dx", float("nan")),
                                         ("dt", 1.0), ("precision", 7), ("tile", 99), ("lambda_", -1.0),
                                         ("lines", 16), ("lines", -1)])
def test_invalid_parameters_are_rejected(field, value):
    from paper_0801_4169_amd import _binding as B
    assert B.fdlb_required_bytes(_sod_params(**{field: value})) == 0


def test_unpaired_periodic_and_equal_speeds_are_rejected():
    from paper_0801_4169_amd import _binding as B
    prm = _sod_params()
    prm.bc[2].kind = B.FDLB_BC_WALL  # y- wall with y+ periodic
    assert B.fdlb_required_bytes(prm) == 0
    prm = _sod_params()
    prm.v[1] = prm.v[0]
    assert B.fdlb_required_bytes(prm) == 0


def test_create_rejects_short_or_misaligned_arena():
    from paper_0801_4169_amd import _binding as B
    prm = _sod_params()
    n = B.fdlb_required_bytes(prm)
    with pytest.raises(B.FdlbError) as e:
        B.fdlb_create(prm, 0, 0x1000, n - 1)
    assert e.value.status == B.FDLB_EINVAL
    with pytest.raises(B.FdlbError):
        B.fdlb_create(prm, 0, 0x1008, n)


def test_strings_and_tile_shapes():
    from paper_0801_4169_amd import _binding as B
    assert "invalid" in B.fdlb_strerror(B.FDLB_EINVAL)
    assert "non-physical" in B.fdlb_strerror(B.FDLB_ENONPHYS)
    shapes = B.fdlb_tile_shapes()
    assert (32, 8) in shapes and all(tx * ty <= 1024 for tx, ty in shapes)


def test_side_segments_are_validated():
    """A lower segment on a periodic side, or with an invalid Dirichlet state, is rejected;
    a valid one is accepted."""
    import fdlb_inputs as fi
    from paper_0801_4169_amd import _binding as B
    prob = fi.problem(40, 20, 1e-3, 1e-6, 2e-6, 2.0, ("dirichlet", "outflow", "wall", "dirichlet"),
                      lower=(None, None, ("dirichlet", (1.0, 0.0, 0.0, 1.0), 0.01, 5.0), None))
    assert B.fdlb_required_bytes(B.make_params(prob)) > 0
    bad = fi.problem(40, 20, 1e-3, 1e-6, 2e-6, 2.0, ("periodic", "periodic", "wall", "dirichlet"),
                     lower=(("wall", (1.0, 0.0, 0.0, 1.0), 0.01, 0.0), None, None, None))
    assert B.fdlb_required_bytes(B.make_params(bad)) == 0
    bad = fi.problem(40, 20, 1e-3, 1e-6, 2e-6, 2.0, ("dirichlet", "outflow", "wall", "dirichlet"),
                     lower=(None, None, ("dirichlet", (-1.0, 0.0, 0.0, 1.0), 0.01, 0.0), None))
    assert B.fdlb_required_bytes(B.make_params(bad)) == 0



def test_binding_uses_one_hip_runtime_whatever_the_import_order():
    """Importing the package before torch still maps a single HIP runtime and a single HSA
    runtime (two HSA runtimes in one process do not share devices or memory)."""
    import subprocess
    import sys
    code = ("import paper_0801_4169_amd, torch\n"
            "m = open('/proc/self/maps').read().splitlines()\n"
            "libs = {l.split()[-1] for l in m if l.split() and l.split()[-1].startswith('/')}\n"
            "print(sum('libamdhip64' in x for x in libs), sum('libhsa-runtime64' in x for x in libs))\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.split()[-2:] == ["1", "1"], r.stdout


def test_failed_create_keeps_no_stale_message():
    """fdlb_last_error(NULL) describes the calling thread's last failed create; a create
    rejected for its arguments leaves it empty."""
    from paper_0801_4169_amd import _binding as B
    prm = _sod_params()
    with pytest.raises(B.FdlbError) as e:
        B.fdlb_create(prm, 0, 0x1000, 1)
    assert e.value.status == B.FDLB_EINVAL
    assert B._lib.fdlb_last_error(None).decode() == ""


def test_largest_planes():
    """A plane holds at most 2^28 cells, and in float64 the row-padded plane (nx rounded up
    to 32) must stay within the 32-bit byte offsets the interior tiles use."""
    from paper_0801_4169_amd import _binding as B
    ok = _sod_params(nx=16384, ny=16383)                      # 2 147 352 576 bytes per plane
    assert B.fdlb_required_bytes(ok) > 0
    assert B.fdlb_required_bytes(_sod_params(nx=16385, ny=16383)) == 0   # padded to 16416
    assert B.fdlb_required_bytes(_sod_params(nx=16385, ny=16383, precision=B.FDLB_F32)) > 0
    assert B.fdlb_required_bytes(_sod_params(nx=1 << 14, ny=(1 << 14) + 1, precision=B.FDLB_F32)) == 0


def test_two_step_passes_take_a_third_buffer_and_float64_only():
    from paper_0801_4169_amd import _binding as B
    one = B.fdlb_required_bytes(_sod_params())
    two = B.fdlb_required_bytes(_sod_params(tblock=2))
    assert two * 2 == one * 3  # three buffer slots instead of two
    assert B.fdlb_required_bytes(_sod_params(tblock=3)) == 0
    assert B.fdlb_required_bytes(_sod_params(tblock=-1)) == 0
    assert B.fdlb_required_bytes(_sod_params(tblock=2, precision=B.FDLB_F32)) == 0
    assert B.fdlb_required_bytes(_sod_params(tblock=2, precision=B.FDLB_F32_DEV)) == 0


def test_frozen_theta_is_validated():
    """theta_fixed is 0 or 1; a frozen theta is finite and non-negative (Sec. 4 freezes theta
    of line IV); an unfrozen context ignores theta_value."""
    from paper_0801_4169_amd import _binding as B
    assert B.fdlb_required_bytes(_sod_params(theta_fixed=1, theta_value=0.7)) > 0
    assert B.fdlb_required_bytes(_sod_params(theta_fixed=1, theta_value=0.0)) > 0
    assert B.fdlb_required_bytes(_sod_params(theta_fixed=0, theta_value=float("nan"))) > 0
    assert B.fdlb_required_bytes(_sod_params(theta_fixed=2, theta_value=0.7)) == 0
    assert B.fdlb_required_bytes(_sod_params(theta_fixed=1, theta_value=-0.1)) == 0
    assert B.fdlb_required_bytes(_sod_params(theta_fixed=1, theta_value=float("inf"))) == 0
    p = B.make_params(__import__("fdlb_inputs").sod_tube()[0], theta=0.25)
    assert p.theta_fixed == 1 and p.theta_value == 0.25
