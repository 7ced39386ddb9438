"""Host-only checks of the C ABI: the library loads, exports every symbol the header
declares, fills defaults, sizes footprints and rejects bad arguments before any
device work (no GPU needed)."""
from __future__ import annotations

import ctypes as C
import re
from pathlib import Path

import pytest

from paper_2505_10168_amd import binding as B

HEADER = Path(__file__).resolve().parent.parent / "include" / "stmg.h"


def declared_functions():
    text = HEADER.read_text()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(stmg_\w+)\s*\(", text, re.M)))


def test_header_declares_and_library_exports_every_entry_point():
    names = declared_functions()
    assert len(names) >= 18
    assert sorted(B.EXPORTED) == names
    lib = C.CDLL(str(B.LIB_PATH))
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layouts_match_header_sizes():
    # field counts of the ctypes mirrors equal the header's struct members
    text = HEADER.read_text()
    for cname, cls in (("stmg_problem", B.stmg_problem), ("stmg_options", B.stmg_options)):
        body = re.search(r"typedef struct \{([^}]*)\}\s*" + cname + ";", text).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        members = [m.strip() for decl in body.split(";") if decl.strip()
                   for m in decl.strip().split(None, 1)[1].split(",")]
        assert [f[0] for f in cls._fields_] == members


def test_default_options():
    o = B.stmg_default_options()
    assert (o.nu, o.omega, o.lambda_crit, o.min_coarse_dofs, o.max_cycles) == (2, 0.5, 0.25, 1024, 100)
    assert (o.tol, o.diverge, o.reassembly, o.precision, o.fused) == (1e-10, 1e9, 0, 0, 1)


def test_footprint_grows_with_grid_and_precision():
    o = B.make_options()
    small = B.stmg_footprint(B.Problem(64, 64).c_struct(), o)
    big = B.stmg_footprint(B.Problem(1024, 4096).c_struct(), o)
    assert big > 20 * small > 0
    # FP64 vectors: at least u, b, t and the load on the fine grid
    assert big >= 4 * 4097 * 1056 * 8
    mixed = B.stmg_footprint(B.Problem(1024, 4096).c_struct(), B.make_options(precision=B.STMG_MIXED))
    assert mixed < big
    fixed = B.stmg_footprint(B.Problem(1024, 4096).c_struct(), B.make_options(deff_mode=1))
    assert fixed <= big


def test_footprint_counts_the_request_outputs():
    """with_adjoint adds the adjoint solution and the gradient to the solution vector."""
    o = B.make_options()
    prob = B.Problem(100, 300)
    f0 = B.stmg_footprint(prob.c_struct(), o, False)
    f1 = B.stmg_footprint(prob.c_struct(), o, True)
    assert f1 - f0 == (101 * 301 + 100) * 8


def test_field_kind_validation():
    """A conductivity field has no densities: reassembly D and the SIMP-extrema D_eff
    need field_kind = density; unknown kinds are rejected."""
    cond = B.Problem(64, 64, field_kind=B.STMG_FIELD_CONDUCTIVITY)
    assert B.stmg_footprint(cond.c_struct(), B.make_options()) > 0
    for bad in (dict(reassembly=B.STMG_REASSEMBLE_D), dict(deff_mode=1)):
        with pytest.raises(B.StmgError) as e:
            B.stmg_footprint(cond.c_struct(), B.make_options(**bad))
        assert e.value.code == B.STMG_EINVAL
    with pytest.raises(B.StmgError) as e:
        B.stmg_footprint(B.Problem(64, 64, field_kind=2).c_struct(), B.make_options())
    assert e.value.code == B.STMG_EINVAL
    with pytest.raises(B.StmgError):
        B.stmg_footprint(B.Problem(64, 64).c_struct(), B.make_options(debug_poison=2))


@pytest.mark.parametrize("field,value", [("n_el", 0), ("n_t", -1), ("length", 0.0),
                                         ("k_ins", -1.0), ("theta_ref", 0.0)])
def test_create_rejects_bad_problem_without_device_work(field, value):
    p = B.Problem(8, 8).c_struct()
    setattr(p, field, value)
    o = B.make_options()
    h = C.c_void_p()
    rc = B.lib.stmg_create(C.byref(h), C.byref(p), C.byref(o), C.c_void_p(1), None, None)
    assert rc == B.STMG_EINVAL and not h.value
    assert B.lib.stmg_last_error()


@pytest.mark.parametrize("field,value", [("nu", -1), ("omega", 0.0), ("max_cycles", 0),
                                         ("max_cycles", 5000), ("precision", 7), ("reassembly", 9),
                                         ("min_coarse_dofs", 0), ("tol", -1.0), ("fused", 3),
                                         ("fused", -1), ("time_kernels", -1), ("interp", 2),
                                         ("time_levels", -1)])
def test_create_rejects_bad_options(field, value):
    p = B.Problem(8, 8).c_struct()
    o = B.make_options(**{field: value})
    h = C.c_void_p()
    rc = B.lib.stmg_create(C.byref(h), C.byref(p), C.byref(o), C.c_void_p(1), None, None)
    assert rc == B.STMG_EINVAL


def test_null_arguments():
    assert B.lib.stmg_default_options(None) == B.STMG_EINVAL
    assert B.lib.stmg_solve_forward(None, None, None, None, None) == B.STMG_EINVAL
    assert B.lib.stmg_objective(None, None, None) == B.STMG_EINVAL
    assert B.lib.stmg_oc_update(None, None, None, 0.5, 0.2, 0.5, 1e-3, None) == B.STMG_EINVAL
    assert B.lib.stmg_destroy(None) == 0
    assert B.lib.stmg_status_string(B.STMG_DIVERGED) == b"diverged"


def test_galerkin_footprint_in_mixed_precision():
    """P in mixed precision is accepted; its footprint counts the FP32 copies of the stored
    stencils and of the coarse vectors, and no FP64 coarse vectors."""
    p = B.Problem(64, 64).c_struct()
    sizes = {}
    for reas in (B.STMG_REASSEMBLE_R, B.STMG_REASSEMBLE_P):
        for prec in (B.STMG_FP64, B.STMG_MIXED):
            o = B.make_options(reassembly=reas, precision=prec, deff_mode=1, max_levels=3)
            n = C.c_size_t()
            assert B.lib.stmg_footprint(C.byref(p), C.byref(o), 0, C.byref(n)) == 0
            sizes[reas, prec] = n.value
    extra64 = sizes[B.STMG_REASSEMBLE_P, B.STMG_FP64] - sizes[B.STMG_REASSEMBLE_R, B.STMG_FP64]
    extra32 = sizes[B.STMG_REASSEMBLE_P, B.STMG_MIXED] - sizes[B.STMG_REASSEMBLE_R, B.STMG_MIXED]
    assert extra32 > 0 and extra64 > 0
    # the FP64 stencils are kept in both; mixed adds their FP32 copy, FP64 a residual vector
    assert extra32 != extra64


def test_footprint_counts_the_bilinear_galerkin_coarsest_factors():
    p = B.Problem(64, 64).c_struct()
    sizes = {}
    for interp in (B.STMG_INTERP_C, B.STMG_INTERP_B):
        o = B.make_options(reassembly=B.STMG_REASSEMBLE_P, interp=interp, deff_mode=1,
                           max_levels=2)
        n = C.c_size_t()
        assert B.lib.stmg_footprint(C.byref(p), C.byref(o), 0, C.byref(n)) == 0
        sizes[interp] = n.value
    assert sizes[B.STMG_INTERP_B] > sizes[B.STMG_INTERP_C] + 2 * (33 * 65) ** 2 * 8 - 1


C_CONSUMER = r"""
#include "stmg.h"
#include <stdio.h>
#include <string.h>
int main(void) {
    stmg_options o;
    stmg_problem p;
    size_t bytes = 0;
    if (stmg_default_options(&o) != STMG_OK) return 1;
    if (stmg_default_options(NULL) != STMG_EINVAL) return 2;
    memset(&p, 0, sizeof p);
    p.n_el = 64; p.n_t = 64; p.length = 1.0; p.t_final = 0.1;
    p.k_ins = 1e-3; p.k_con = 1.0; p.c_ins = 1.0; p.c_con = 1.0; p.p_k = 3.0; p.p_c = 2.0;
    p.theta_ref = 1.0; p.q_uniform = 1.0;
    if (stmg_footprint(&p, &o, 1, &bytes) != STMG_OK || bytes == 0) return 3;
    if (stmg_create(NULL, &p, &o, NULL, NULL, NULL) != STMG_EINVAL) return 4;
    printf("%s %zu %d\n", stmg_status_string(STMG_DIVERGED), bytes, o.nu);
    return 0;
}
"""


def test_header_compiles_as_c99_and_links(tmp_path):
    """A plain C99 program compiles against include/stmg.h with warnings as errors,
    links against libstmg.so and calls the entry points that need no GPU."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "consumer.c"
    src.write_text(C_CONSUMER)
    exe = tmp_path / "consumer"
    lib = B.LIB_PATH.parent
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                    f"-I{HEADER.parent}", str(src), f"-L{lib}", "-lstmg",
                    f"-Wl,-rpath,{lib}", "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert out[0] == "diverged" and int(out[1]) > 0 and int(out[2]) == 2


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes mirror of a header struct has the C compiler's size and field
    offsets, so a field added on one side only fails here rather than in a solve."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    mirrors = [B.stmg_problem, B.stmg_options, B.stmg_stats, B.stmg_info]
    lines = []
    for st in mirrors:
        name = st.__name__
        lines.append(f'printf("{name} sizeof %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "stmg.h"\n'
                   "int main(void) {\n" + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", f"-I{HEADER.parent}", str(src),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        sname, fname, val = line.split()
        got[sname, fname] = int(val)
    for st in mirrors:
        name = st.__name__
        assert got[name, "sizeof"] == C.sizeof(st), name
        for f, _ in st._fields_:
            assert got[name, f] == getattr(st, f).offset, (name, f)


@pytest.mark.parametrize("n_el,n_t,sweeps,fp32,fine", [
    (8192, 65536, 2, 0, 1), (8192, 65536, 4, 0, 1), (4096, 65536, 2, 1, 1), (1024, 4096, 5, 0, 1),
    (512, 2048, 5, 0, 0), (64, 64, 5, 0, 0), (7, 128, 2, 0, 0), (3, 5, 6, 1, 0)])
def test_pass_geometry_covers_the_level(n_el, n_t, sweeps, fp32, fine):
    """The launch geometry of a fused pass (host-only): the useful strips cover every
    node column, the halo is at least the chain's reach on each side and keeps the
    useful strip a whole number of 128-byte lines, the time segments are even (a t
    restriction pairs levels inside one segment) and cover every time level, and the
    wavefront count is strips x segments."""
    g = B.stmg_pass_geometry(n_el, n_t, sweeps, bool(fp32), bool(fine))
    k = 4 if fp32 else 2                       # columns per lane (16 bytes)
    u, xw, seg, waves = g["strip_cols"], g["strips"], g["seg_rows"], g["waves"]
    halo_lanes = (64 - u // k) // 2
    assert u % k == 0 and halo_lanes * k >= sweeps + 2
    assert (u * (8 if not fp32 else 4)) % 128 == 0
    assert xw * u >= n_el + 1 > (xw - 1) * u
    assert seg >= 2 and seg % 2 == 0
    assert waves == xw * -(-(n_t + 1) // seg)
