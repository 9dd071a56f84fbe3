"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and rejects invalid arguments before touching a device."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mb4.h")

from paper_2003_04345_amd import mb4 as M  # noqa: E402


def _declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"MB4_API\s+[^;]*?\b(mb4_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(M.LIB_PATH):
        pytest.fail("libmb4.so is not built; run __graft_entry__.build()")
    return M.load_library()


def test_header_declares_the_boundary():
    names = _declared_symbols()
    for required in ("mb4_create", "mb4_step", "mb4_energy", "mb4_destroy",
                     "mb4_newton_update", "mb4_stage_solve"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_symbols():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", M.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert exported == set(_declared_symbols())


def test_header_compiles_as_c():
    # The boundary is plain C: the header must compile with a C compiler.
    src = '#include "mb4.h"\nint main(void){mb4_options o; mb4_options_default(&o); return 0;}\n'
    res = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only",
                          f"-I{os.path.dirname(HEADER)}", "-x", "c", "-"],
                         input=src, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr


def test_struct_layout_matches_binding():
    # Offsets the C compiler assigns, against the ctypes mirror.
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "mb4.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(mb4_lattice), offsetof(mb4_lattice, t_hop),
         offsetof(mb4_lattice, diag_shift), sizeof(mb4_nonlinearity));
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(mb4_options), offsetof(mb4_options, max_newton),
         offsetof(mb4_options, inner_sweeps), offsetof(mb4_options, stream),
         offsetof(mb4_options, mem_budget), offsetof(mb4_options, flags));
  return 0;
}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "layout")
        res = subprocess.run(["gcc", "-std=c99", f"-I{os.path.dirname(HEADER)}", "-x", "c", "-",
                              "-o", exe], input=prog, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    a = [int(x) for x in lines[0].split()]
    b = [int(x) for x in lines[1].split()]
    assert a == [ctypes.sizeof(M.mb4_lattice), M.mb4_lattice.t_hop.offset,
                 M.mb4_lattice.diag_shift.offset, ctypes.sizeof(M.mb4_nonlinearity)]
    assert b == [ctypes.sizeof(M.mb4_options), M.mb4_options.max_newton.offset,
                 M.mb4_options.inner_sweeps.offset, M.mb4_options.stream.offset,
                 M.mb4_options.mem_budget.offset, M.mb4_options.flags.offset]


def _create(lat=None, v=None, g=1.0, h=0.01, opt=None):
    lib = M.load_library()
    lat = lat if lat is not None else M.mb4_lattice(8, 8, 1.0, 0.0)
    n = max(lat.nx * lat.ny, 1)
    v = v if v is not None else np.zeros(n)
    out = ctypes.c_void_p(1234)
    rc = lib.mb4_create(ctypes.byref(lat), v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        ctypes.byref(M.mb4_nonlinearity(g)), h,
                        ctypes.byref(opt) if opt is not None else None, ctypes.byref(out))
    return rc, out


@pytest.mark.parametrize("kwargs", [
    dict(lat=M.mb4_lattice(2, 8, 1.0, 0.0)),
    dict(lat=M.mb4_lattice(8, 2, 1.0, 0.0)),
    dict(lat=M.mb4_lattice(1 << 15, 1 << 14, 1.0, 0.0), v=np.zeros(1)),
    dict(lat=M.mb4_lattice(8, 8, float("nan"), 0.0)),
    dict(lat=M.mb4_lattice(8, 8, 1.0, float("inf"))),
    dict(g=float("nan")),
    dict(h=0.0),
    dict(h=float("inf")),
    dict(v=np.array([0.0] * 63 + [float("nan")])),
])
def test_create_rejects_invalid_arguments(lib, kwargs):
    rc, out = _create(**kwargs)
    assert rc == M.MB4_EINVAL
    assert out.value is None
    assert M.error_detail() != ""


@pytest.mark.parametrize("field,value", [("eps", -1.0), ("eps", float("nan")), ("eps", 1.0),
                                         ("max_newton", -1), ("max_newton", 1001),
                                         ("inner_sweeps", -2), ("inner_sweeps", 65),
                                         ("flags", 16), ("flags", 0x80000000)])
def test_create_rejects_invalid_options(lib, field, value):
    opt = M.mb4_options_default()
    setattr(opt, field, value)
    rc, _ = _create(opt=opt)
    assert rc == M.MB4_EINVAL


def test_memory_budget_is_enforced_before_allocation(lib):
    opt = M.mb4_options_default()
    opt.mem_budget = 1000   # far below 264 bytes/site * 64 sites
    rc, out = _create(opt=opt)
    assert rc == M.MB4_ENOMEM
    assert out.value is None


def test_null_arguments(lib):
    assert lib.mb4_create(None, None, None, 0.01, None, None) == M.MB4_EINVAL
    lat = M.mb4_lattice(8, 8, 1.0, 0.0)
    out = ctypes.c_void_p()
    assert lib.mb4_create(ctypes.byref(lat), None, ctypes.byref(M.mb4_nonlinearity(1.0)), 0.01,
                          None, ctypes.byref(out)) == M.MB4_EINVAL
    assert lib.mb4_step(None, 1) == M.MB4_EINVAL
    assert lib.mb4_energy(None, None) == M.MB4_EINVAL
    assert lib.mb4_set_state(None, None, None) == M.MB4_EINVAL
    assert lib.mb4_set_h(None, 0.1) == M.MB4_EINVAL
    assert lib.mb4_steps_done(None) == -1
    assert lib.mb4_last_stats(None, None, None, None) == M.MB4_EINVAL
    assert lib.mb4_newton_update(None, None, None, None, None) == M.MB4_EINVAL
    assert lib.mb4_stage_solve(None, None, None, 1) == M.MB4_EINVAL
    assert lib.mb4_set_region(None, 0) == M.MB4_EINVAL
    assert lib.mb4_region(None) == -1
    assert lib.mb4_set_sweeps(None, 3) == M.MB4_EINVAL
    assert lib.mb4_sweeps(None) == -1
    assert lib.mb4_tune(None, 4, None, None, None) == M.MB4_EINVAL
    lib.mb4_destroy(None)


def test_options_default_values(lib):
    o = M.mb4_options_default()
    assert o.eps == 1e-13 and o.max_newton == 50 and o.inner_sweeps == 3
    assert o.stream is None and o.mem_budget == 0 and o.flags == 0


def test_strerror_covers_codes(lib):
    for code in (M.MB4_OK, M.MB4_EINVAL, M.MB4_ENOMEM, M.MB4_EDEVICE, M.MB4_ENOCONV):
        assert M.strerror(code)
    assert "unknown" in M.strerror(12345)


def test_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(FileNotFoundError):
        M.load_library(str(tmp_path / "libmb4.so"))


def test_constants_header_is_up_to_date():
    gen = os.path.join(ROOT, "paper_2003_04345_amd", "csrc", "gen_constants.py")
    res = subprocess.run([sys.executable, gen, "--check"], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr


def _header_constants():
    text = open(os.path.join(ROOT, "paper_2003_04345_amd", "csrc", "mb4_constants.h")).read()
    out = {}
    for m in re.finditer(r"static constexpr double (\w+)(\[[^=]*\])\s*=\s*\{(.*?)\};", text, re.S):
        name, dims, body = m.group(1), m.group(2), m.group(3)
        vals = [float.fromhex(x.strip()) if "0x" in x else float(x)
                for x in re.sub(r"[{}\s]", " ", body).replace(" ", "").split(",") if x]
        shape = [int(d) for d in re.findall(r"\[(\d+)\]", dims)]
        out[name] = np.array(vals).reshape(shape)
    return out


def test_gpu_constants_agree_with_the_oracle():
    # Two independent derivations (sympy for the library, exact fractions
    # plus numpy for the oracle) of the same constants.
    import oracle as O
    k = O.method_constants()
    c = _header_constants()
    np.testing.assert_array_equal(c["MB4_E"], k.E)
    np.testing.assert_array_equal(c["MB4_E0"], k.E_full[:, 0])
    np.testing.assert_allclose(c["MB4_LAMBDA"], k.lam, rtol=0, atol=1e-14)
    # Eigenvectors are fixed up to sign (both sides use unit columns); the
    # Newton root does not depend on their scaling.
    sign = np.sign(k.T[0, :])
    np.testing.assert_allclose(c["MB4_T"], k.T * sign[None, :], rtol=0, atol=1e-14)
    np.testing.assert_allclose(c["MB4_TINV"], k.Tinv * sign[:, None], rtol=0, atol=1e-14)


def test_gauss_legendre_tables_reproduce_E_and_the_cubic_integrals():
    import oracle as O
    k = O.method_constants()
    c = _header_constants()
    q, lq = c["MB4_GL_Q"], c["MB4_GL_L"]
    np.testing.assert_allclose(q @ lq, k.E_full, rtol=0, atol=1e-13)
    # Six nodes integrate A_{c_i,z} l_a l_b l_d (degree 11) exactly ...
    cub6 = np.einsum("iq,qa,qb,qd->iabd", q, lq, lq, lq)
    np.testing.assert_allclose(cub6, k.cubic, rtol=0, atol=1e-12)
    # ... and a 5-node rule does not (negative control): stages 1 and 2 fail.
    x, w = np.polynomial.legendre.leggauss(5)
    z, w = (x + 1) / 2, w / 2
    from fractions import Fraction
    from oracle.mb4_oracle import a_of_tau, lagrange_basis
    nodes = [Fraction(0)] + list(O.C_PAPER)
    ell = lagrange_basis(nodes)
    l5 = np.array([[sum(float(cf) * zz ** p for p, cf in enumerate(ell[j])) for j in range(4)]
                   for zz in z])
    a5 = np.array([[w[qq] * sum(float(cf) * z[qq] ** p
                                for p, cf in enumerate(a_of_tau(nodes[i + 1], O.ALPHA1_PAPER)))
                    for qq in range(5)] for i in range(3)])
    cub5 = np.einsum("iq,qa,qb,qd->iabd", a5, l5, l5, l5)
    err = np.max(np.abs(cub5 - k.cubic), axis=(1, 2, 3))
    assert err[0] > 1e-6 and err[1] > 1e-6 and err[2] < 1e-12


def _ens_create(lib, count=2, lats=None, pots=None, gs=None, hs=None, opt=None,
                null=None):
    lats = lats if lats is not None else [M.mb4_lattice(8, 8, 1.0, 0.0)] * count
    pots = pots if pots is not None else [np.zeros(l.nx * l.ny) for l in lats]
    gs = gs if gs is not None else [1.0] * len(lats)
    hs = hs if hs is not None else [0.01] * len(lats)
    n = len(lats)
    c_lats = (M.mb4_lattice * max(n, 1))(*lats)
    c_pots = (ctypes.POINTER(ctypes.c_double) * max(n, 1))(
        *[p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if p is not None else None
          for p in pots])
    c_nls = (M.mb4_nonlinearity * max(n, 1))(*[M.mb4_nonlinearity(g) for g in gs])
    c_h = (ctypes.c_double * max(n, 1))(*hs)
    args = [count, c_lats, c_pots, c_nls, c_h]
    if null is not None:
        args[null] = None
    out = ctypes.c_void_p(1234)
    rc = lib.mb4_ensemble_create(*args, ctypes.byref(opt) if opt is not None else None,
                                 ctypes.byref(out))
    return rc, out


@pytest.mark.parametrize("case", [
    dict(count=0, lats=[]),
    dict(count=65537),
    dict(null=1), dict(null=2), dict(null=3), dict(null=4),
    dict(lats=[M.mb4_lattice(8, 8, 1.0, 0.0), M.mb4_lattice(2, 8, 1.0, 0.0)]),
    dict(lats=[M.mb4_lattice(8, 8, float("nan"), 0.0), M.mb4_lattice(8, 8, 1.0, 0.0)]),
    dict(gs=[1.0, float("inf")]),
    dict(hs=[0.01, 0.0]),
    dict(pots=[np.zeros(64), np.array([0.0] * 63 + [float("nan")])]),
    dict(pots=[np.zeros(64), None]),
])
def test_ensemble_create_rejects_invalid_arguments(lib, case):
    rc, out = _ens_create(lib, **case)
    assert rc == M.MB4_EINVAL
    assert out.value is None
    assert M.error_detail() != ""


@pytest.mark.parametrize("field,value", [("inner_sweeps", 5), ("eps", -1.0),
                                         ("max_newton", 1001), ("flags", 8)])
def test_ensemble_create_rejects_invalid_options(lib, field, value):
    opt = M.mb4_options_default()
    setattr(opt, field, value)
    rc, _ = _ens_create(lib, opt=opt)
    assert rc == M.MB4_EINVAL


def test_ensemble_memory_budget_is_enforced_before_allocation(lib):
    opt = M.mb4_options_default()
    opt.mem_budget = 4096   # below 136 bytes/site * 128 sites
    rc, out = _ens_create(lib, opt=opt)
    assert rc == M.MB4_ENOMEM
    assert out.value is None


def test_ensemble_calls_reject_null(lib):
    assert lib.mb4_ensemble_step(None, 1) == M.MB4_EINVAL
    assert lib.mb4_ensemble_set_state(None, 0, None, None) == M.MB4_EINVAL
    assert lib.mb4_ensemble_get_state(None, 0, None, None) == M.MB4_EINVAL
    assert lib.mb4_ensemble_energy_components(None, None) == M.MB4_EINVAL
    assert lib.mb4_ensemble_member_stats(None, 0, None, None) == M.MB4_EINVAL
    assert lib.mb4_ensemble_set_region(None, 0) == M.MB4_EINVAL
    assert lib.mb4_ensemble_tune(None, 1, None, None) == M.MB4_EINVAL
    assert lib.mb4_ensemble_tune_all(None, 1, None, None, None) == M.MB4_EINVAL
    assert lib.mb4_ensemble_set_sweeps(None, 3) == M.MB4_EINVAL
    assert lib.mb4_ensemble_size(None) == -1
    assert lib.mb4_ensemble_region(None) == -1
    assert lib.mb4_ensemble_sweeps(None) == -1
    lib.mb4_ensemble_destroy(None)


def test_fp32_solves_take_at_most_four_sweeps(lib):
    opt = M.mb4_options_default()
    opt.flags = M.MB4_FLAG_FP32_SOLVE
    opt.inner_sweeps = 5
    rc, out = _create(opt=opt)
    assert rc == M.MB4_EINVAL and out.value is None


def test_spectral_solves_are_fp64_and_limited_in_size(lib):
    opt = M.mb4_options_default()
    opt.flags = M.MB4_FLAG_SPECTRAL_SOLVE | M.MB4_FLAG_FP32_SOLVE
    rc, out = _create(opt=opt)
    assert rc == M.MB4_EINVAL and out.value is None
    assert "FP64" in M.error_detail()
    opt.flags = M.MB4_FLAG_SPECTRAL_SOLVE
    for lat in (M.mb4_lattice(1025, 4, 1.0, 0.0), M.mb4_lattice(4, 1025, 1.0, 0.0)):
        rc, out = _create(lat=lat, opt=opt)
        assert rc == M.MB4_EINVAL and out.value is None
        assert "1024" in M.error_detail()


def test_spectral_flag_is_for_single_states(lib):
    opt = M.mb4_options_default()
    opt.flags = M.MB4_FLAG_SPECTRAL_SOLVE
    lats = (M.mb4_lattice * 1)(M.mb4_lattice(8, 8, 1.0, 0.0))
    nls = (M.mb4_nonlinearity * 1)(M.mb4_nonlinearity(1.0))
    v = np.zeros(64)
    pots = (ctypes.POINTER(ctypes.c_double) * 1)(v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    hs = (ctypes.c_double * 1)(0.01)
    out = ctypes.c_void_p(1234)
    rc = lib.mb4_ensemble_create(1, lats, pots, nls, hs, ctypes.byref(opt), ctypes.byref(out))
    assert rc == M.MB4_EINVAL and "single states" in M.error_detail()
    srv = ctypes.c_void_p(1234)
    rc = lib.mb4_server_create(1 << 26, 4, 4, ctypes.byref(opt), ctypes.byref(srv))
    assert rc == M.MB4_EINVAL and "single states" in M.error_detail()


def test_server_struct_layouts_match_binding():
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "mb4.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(mb4_request_info),
         offsetof(mb4_request_info, steps), offsetof(mb4_request_info, steps_done),
         offsetof(mb4_request_info, t_submit), offsetof(mb4_request_info, energy_start),
         offsetof(mb4_request_info, energy_end), offsetof(mb4_request_info, last_newton_iters),
         offsetof(mb4_request_info, error));
  printf("%zu %zu %zu %zu %zu\n", sizeof(mb4_server_info), offsetof(mb4_server_info, queued),
         offsetof(mb4_server_info, active), offsetof(mb4_server_info, batches),
         offsetof(mb4_server_info, site_steps));
  return 0;
}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "layout")
        res = subprocess.run(["gcc", "-std=c99", f"-I{os.path.dirname(HEADER)}", "-x", "c", "-",
                              "-o", exe], input=prog, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    a = [int(x) for x in lines[0].split()]
    b = [int(x) for x in lines[1].split()]
    R, S = M.mb4_request_info, M.mb4_server_info
    assert a == [ctypes.sizeof(R), R.steps.offset, R.steps_done.offset, R.t_submit.offset,
                 R.energy_start.offset, R.energy_end.offset, R.last_newton_iters.offset,
                 R.error.offset]
    assert b == [ctypes.sizeof(S), S.queued.offset, S.active.offset, S.batches.offset,
                 S.site_steps.offset]


@pytest.mark.parametrize("arena,max_active,batch,field,value", [
    (1 << 30, 0, 8, None, None),
    (1 << 30, 65537, 8, None, None),
    (1 << 30, 16, 0, None, None),
    (1 << 30, 16, 33, None, None),
    (1 << 20, 16, 8, None, None),           # arena too small for anything
    (1 << 30, 16, 8, "inner_sweeps", 5),
    (1 << 30, 16, 8, "flags", 8),
    (1 << 30, 16, 8, "eps", float("nan")),
])
def test_server_create_rejects_invalid_arguments(lib, arena, max_active, batch, field, value):
    opt = M.mb4_options_default()
    if field is not None:
        setattr(opt, field, value)
    out = ctypes.c_void_p(1234)
    rc = lib.mb4_server_create(arena, max_active, batch, ctypes.byref(opt), ctypes.byref(out))
    assert rc == M.MB4_EINVAL
    assert out.value is None


def test_server_calls_reject_null(lib):
    assert lib.mb4_server_poll(None, None, None) == M.MB4_EINVAL
    assert lib.mb4_server_submit(None, None, None, None, 0.01, None, None, 1, None) == M.MB4_EINVAL
    assert lib.mb4_server_request(None, 1, None) == M.MB4_EINVAL
    assert lib.mb4_server_result(None, 1, None, None) == M.MB4_EINVAL
    assert lib.mb4_server_release(None, 1) == M.MB4_EINVAL
    assert lib.mb4_server_stats(None, None) == M.MB4_EINVAL
    assert lib.mb4_server_clock(None) == -1.0
    lib.mb4_server_destroy(None)


def test_noalloc_energy_validates_before_any_device_call(lib):
    # Non-NULL stand-ins for device pointers: every call below is rejected on
    # the host, so none of them is dereferenced.
    fake = ctypes.c_void_p(256)
    nl = M.mb4_nonlinearity(1.0)

    def call(lat, nonlin=nl, ptrs=(fake, fake, fake, fake)):
        return lib.mb4_energy_components_noalloc(
            ctypes.byref(lat) if lat is not None else None,
            ctypes.byref(nonlin) if nonlin is not None else None, *ptrs, None)

    ok = M.mb4_lattice(64, 64, 1.0, 0.0)
    assert call(None) == M.MB4_EINVAL
    assert call(ok, nonlin=None) == M.MB4_EINVAL
    for k in range(4):
        ptrs = [fake] * 4
        ptrs[k] = None
        assert call(ok, ptrs=tuple(ptrs)) == M.MB4_EINVAL
    assert call(M.mb4_lattice(2, 64, 1.0, 0.0)) == M.MB4_EINVAL
    assert call(M.mb4_lattice(64, 64, float("nan"), 0.0)) == M.MB4_EINVAL
    assert call(ok, nonlin=M.mb4_nonlinearity(float("inf"))) == M.MB4_EINVAL
    # One tile row beyond the 32768 tiles of the scratch array (2048 x 4096
    # is exactly 32768 tiles of 64 x 4).
    assert call(M.mb4_lattice(2048, 4100, 1.0, 0.0)) == M.MB4_EINVAL
    assert "scratch" in M.error_detail()
    assert call(M.mb4_lattice(2049, 4096, 1.0, 0.0)) == M.MB4_EINVAL


def test_set_nonlinearity_sites_rejects_a_null_state(lib):
    g = (ctypes.c_double * 9)(*([1.0] * 9))
    assert lib.mb4_set_nonlinearity_sites(None, g) == M.MB4_EINVAL
