"""The C ABI without a GPU: the library loads, exports every declared entry
point, validates arguments before touching the device, and its parameter
rule stays within the oracle's error budget (written independently)."""
import ctypes
import os
import re

import pytest

import paper_2606_20863_amd as md
from oracle import exact as ox

import rulecheck

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdgemm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(md_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = md.lib()
    names = declared_functions()
    assert "md_gemm" in names and "md_gemm_ex" in names
    for name in names:
        assert hasattr(L, name), name


def test_version_and_strerror():
    L = md.lib()
    assert L.md_version() >= 100
    for code in range(9):
        assert len(L.md_strerror(code)) > 0
    assert L.md_strerror(12345) == b"unknown error"


def test_argument_errors_before_device_work():
    L = md.lib()
    p = ctypes.c_void_p(0x1000)
    # m outside {2, 4, 8}
    assert L.md_gemm(3, 4, 4, 4, p, p, p, None) == 1
    # negative sizes
    assert L.md_gemm(2, -1, 4, 4, p, p, p, None) == 2
    # empty output: no-op success, even with NULL pointers
    assert L.md_gemm(2, 0, 4, 4, None, None, None, None) == 0
    assert L.md_gemm(2, 4, 0, 4, None, None, None, None) == 0
    # NULL data pointers
    assert L.md_gemm(2, 4, 4, 4, None, p, p, None) == 3
    # C overlapping A
    a = ctypes.c_void_p(0x100000)
    c = ctypes.c_void_p(0x100000 + 8)
    b = ctypes.c_void_p(0x900000)
    assert L.md_gemm(2, 4, 4, 4, a, b, c, None) == 4
    # bad leading dimension
    opts = md.MDOpts()
    assert L.md_gemm_ex(2, 0, 0, 4, 4, 4, a, 3, 16, b, 4, 16, ctypes.c_void_p(0x500000), 4, 16,
                        ctypes.byref(opts), None) == 2
    # unknown form
    opts.form = 9
    assert L.md_gemm_ex(2, 0, 0, 4, 4, 4, a, 4, 16, b, 4, 16, ctypes.c_void_p(0x500000), 4, 16,
                        ctypes.byref(opts), None) == 7
    # forced INT8 slices must be 7 bits wide
    opts.form = 1
    opts.force_S = 8
    opts.force_beta = 9
    assert L.md_gemm_ex(2, 0, 0, 4, 4, 4, a, 4, 16, b, 4, 16, ctypes.c_void_p(0x500000), 4, 16,
                        ctypes.byref(opts), None) == 7


def test_dot_argument_errors_before_device_work():
    L = md.lib()
    p = ctypes.c_void_p(0x1000)
    x = ctypes.c_void_p(0x100000)
    y = ctypes.c_void_p(0x900000)
    o = ctypes.c_void_p(0x500000)
    # m outside {1, 2, 4, 8, 16}
    for m in (0, 3, 5, 32):
        assert L.md_dot(m, 4, 4, p, p, p, None) == 1
    # negative sizes; empty batch is a no-op even with NULL pointers
    assert L.md_dot(2, -1, 4, p, p, p, None) == 2
    assert L.md_dot(16, 0, 4, None, None, None, None) == 0
    # NULL data
    assert L.md_dot(2, 4, 4, None, y, o, None) == 3
    # output overlapping X
    assert L.md_dot(2, 4, 4, x, y, ctypes.c_void_p(0x100000 + 8), None) == 4
    # leading dimension below n, output planes closer than the batch
    opts = md.MDOpts()
    assert L.md_dot_ex(2, 4, 8, x, 7, 32, y, 8, 32, o, 4, ctypes.byref(opts), None) == 2
    assert L.md_dot_ex(2, 4, 8, x, 8, 32, y, 8, 32, o, 3, ctypes.byref(opts), None) == 2
    # no debug dump for inner products
    dbg = md.MDDebug()
    opts.dbg = ctypes.pointer(dbg)
    assert L.md_dot_ex(2, 4, 8, x, 8, 32, y, 8, 32, o, 4, ctypes.byref(opts), None) == 7


@pytest.mark.parametrize("form", ["int8", "int8bal", "fp64"])
@pytest.mark.parametrize("K", [1, 64, 100, 1024, 2048, 4096, 100000])
@pytest.mark.parametrize("T,G", [(100, 2), (100, 40), (200, 3), (200, 44), (400, 9), (400, 34)])
def test_parameter_rule_against_budget(form, K, T, G):
    """md_choose_params against the oracle's error budget: at least the
    budget's slices and fewer than one band more, every accumulation exact,
    the chunk as deep as exactness and K allow (to a granule).  The library
    refuses only where not even one fragment's depth is exact."""
    try:
        beta, S, kc, band = md.choose_params(form, K, T, G)
    except md.MDError:
        beta = 7 if form == "int8" else 8
        if form == "fp64":
            assert all(ox.exact_depth(form, b, ox.min_slices(form, T, G, b)) < rulecheck.GRAN[form]
                       for b in ox.FP64_BETAS)
        else:
            assert ox.exact_depth(form, beta, ox.min_slices(form, T, G)) < rulecheck.GRAN[form]
        return
    rulecheck.check_params(form, K, T, G, beta, S, kc, band)


@pytest.mark.parametrize("form", ["int8", "int8bal", "fp64"])
def test_parameter_rule_sweep(form):
    """The slice count over a dense grid of targets and ratio exponents (the
    searches start at a lower bound of the answer): within the budget's
    rule at every point, equal to its minimum wherever one band holds it."""
    for T in range(1, 900, 13):
        for G in range(0, 260, 7):
            try:
                beta, S, kc, band = md.choose_params(form, 64, T, G)
            except md.MDError:
                continue
            rulecheck.check_params(form, 64, T, G, beta, S, kc, band)


def test_parameter_rule_headline():
    """The benchmark's parameters: quad-double, depth 4096, G = 3 (the
    magnitude certificate of its U(-1,1) inputs)."""
    assert md.choose_params("int8bal", 4096, 200, 3) == (8, 27, 4096, 27)
    assert md.choose_params("int8", 4096, 200, 3) == (7, 30, 4096, 30)
    assert ox.min_slices("int8bal", 200, 3) == 27 and ox.min_slices("int8", 200, 3) == 30


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: --gpus above 1 exits with status 2 and a
    message, before touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU only" in res.stderr


def test_bench_defers_the_error_check_to_the_cpu_leg():
    """bench.py keeps sampled outputs during the GPU runs and checks them
    with the oracle only in its CPU leg: an exact product reads as the
    floor 2^-1074, a perturbed sampled entry as a large error."""
    import sys
    import numpy as np
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench
    r = np.random.Generator(np.random.PCG64(3))
    A = r.integers(1, 8, (1, 10, 12)).astype(np.float64)
    B = r.integers(1, 8, (1, 12, 9)).astype(np.float64)
    C = (A[0] @ B[0])[None]
    C2 = C.copy()
    C2[0, 0, 0] += 1.0
    t, u = {}, {}
    bench.defer_error(t, "err", A, B, C, n=4)
    bench.defer_error(u, "err", A, B, C2, n=4)
    assert t["err"] is None and u["err"] is None
    bench.resolve_errors()
    assert t["err"] == -1074.0
    assert -12 < u["err"] < 0
    assert not bench._ERROR_CHECKS


def test_fixed_limbs_hold_the_largest_sums():
    """md_fixed_limbs against the largest integer a depth-K product can
    reach: every digit at its largest magnitude (sign-magnitude INT8 127,
    balanced -128, FP64 digits 2^beta - 1), so D_t = (t+1) K dmax^2 and X
    = sum_t D_t 2^(beta (S-1-t)) must fit the limbs in two's complement."""
    L = md.lib()
    for beta, dmax in ((7, 127), (8, 128), (12, (1 << 12) - 1), (24, (1 << 24) - 1)):
        for S in (1, 2, 5, 27, 64, 200):
            for K in (1, 3, 1000, 1 << 20, (1 << 31) + 5):
                n = L.md_fixed_limbs(beta, S, K)
                X = K * dmax * dmax * sum((t + 1) << (beta * (S - 1 - t)) for t in range(S))
                ox.fixed_limbs(X, n)
                ox.fixed_limbs(-X, n)
                # and no more than two limbs of slack
                assert n <= 2 or X >= 1 << (32 * (n - 2) - 1), (beta, S, K, n)
    assert L.md_fixed_limbs(0, 4, 10) == -1 and L.md_fixed_limbs(8, 0, 10) == -1
    assert L.md_fixed_limbs(8, 513, 10) == -1 and L.md_fixed_limbs(8, 4, -1) == -1
    assert md.fixed_limbs(8, 27, 4096) == L.md_fixed_limbs(8, 27, 4096)


def test_fixed_argument_errors_before_device_work():
    L = md.lib()
    a = ctypes.c_void_p(0x100000)
    b = ctypes.c_void_p(0x900000)
    x = ctypes.c_void_p(0x500000)
    sc = ctypes.c_void_p(0x700000)
    opts = md.MDOpts()
    opts.form = 2
    opts.force_S = 4
    opts.force_beta = 8
    n = L.md_fixed_limbs(8, 4, 16)

    def gf(m=2, M=4, N=4, K=16, nl=n, X=x, S=sc, o=opts):
        return L.md_gemm_fixed(m, M, N, K, a, K, M * K, b, N, K * N, None, None, X, nl, S,
                               ctypes.byref(o) if o is not None else None, None)

    assert gf(m=3) == 1
    assert gf(o=None) == 7
    unforced = md.MDOpts()
    assert gf(o=unforced) == 7
    assert gf(K=0) == 2
    assert gf(M=0) == 0 and gf(N=0) == 0
    assert gf(nl=n - 1) == 8 and gf(nl=81) == 8
    assert gf(X=None) == 3
    assert gf(S=ctypes.c_void_p(0x500000 + 4 * 16)) == 4       # scale inside X's limbs
    dbg_opts = md.MDOpts()
    dbg_opts.form, dbg_opts.force_S, dbg_opts.force_beta = 2, 4, 8
    dbg = md.MDDebug()
    dbg_opts.dbg = ctypes.pointer(dbg)
    assert gf(o=dbg_opts) == 7
    # exponents: nothing to do, bad sizes, NULL data
    assert L.md_exponents(0, 0, 4, None, 4, None, 4, None, None, None) == 0
    assert L.md_exponents(4, 4, 4, a, 4, b, 4, None, None, None) == 0
    assert L.md_exponents(-1, 4, 4, a, 4, b, 4, x, sc, None) == 2
    assert L.md_exponents(4, 4, 4, None, 4, b, 4, x, None, None) == 3
    assert L.md_exponents(4, 4, 8, a, 4, b, 4, x, None, None) == 2      # lda < K
    # add and round
    assert L.md_fixed_add(-1, 4, x, x, x, None) == 2
    assert L.md_fixed_add(16, 0, x, x, x, None) == 8
    assert L.md_fixed_add(0, 4, None, None, None, None) == 0
    assert L.md_fixed_add(16, 4, None, x, x, None) == 3
    c = ctypes.c_void_p(0x300000)
    assert L.md_fixed_round(3, 16, 4, x, sc, c, 16, None) == 1
    assert L.md_fixed_round(2, 16, 81, x, sc, c, 16, None) == 8
    assert L.md_fixed_round(2, 16, 4, x, sc, c, 15, None) == 2
    assert L.md_fixed_round(2, 16, 4, x, sc, ctypes.c_void_p(0x500000 + 64), 16, None) == 4
    assert L.md_fixed_round(2, 0, 4, None, None, None, 0, None) == 0


def test_plane_layout_of_views():
    """The binding passes a view's own strides (a depth block of larger
    planes addresses the parent in place) and refuses broadcast or
    transposed views, whose dense reading would leave the view."""
    import torch
    x = torch.zeros(2, 3, 5, dtype=torch.float64)
    lay = lambda t: md._plane_layout(tuple(t.shape), tuple(t.stride()))
    assert lay(x) == (5, 15)
    assert lay(x[:, :, 1:4]) == (5, 15)
    assert lay(x[:, 1:, :]) == (5, 15)
    assert lay(x[:1]) == (5, 15) and lay(x[:, :1, :]) == (5, 15)
    with pytest.raises(ValueError):
        lay(torch.zeros(5, dtype=torch.float64).expand(2, 3, 5))
    with pytest.raises(ValueError):
        lay(torch.zeros(3, 5, dtype=torch.float64).expand(2, 3, 5))
    with pytest.raises(ValueError):
        lay(x.transpose(1, 2))


def test_debug_dumps_sized_by_S_need_a_forced_S():
    """Digit and diagonal-sum dumps are sized by S: with the rule choosing S
    the call refuses them before any device work."""
    L = md.lib()
    a = ctypes.c_void_p(0x100000)
    b = ctypes.c_void_p(0x900000)
    opts = md.MDOpts()
    dbg = md.MDDebug()
    dbg.D = 0x700000
    opts.dbg = ctypes.pointer(dbg)
    assert L.md_gemm_ex(2, 0, 0, 4, 4, 4, a, 4, 16, b, 4, 16, ctypes.c_void_p(0x500000), 4, 16,
                        ctypes.byref(opts), None) == 7


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures against the header compiled by gcc:
    size and every field's offset."""
    import subprocess
    structs = {"md_info": md.MDInfo, "md_debug": md.MDDebug, "md_opts": md.MDOpts, "md_cert": md.MDCert}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_workspace_size_names():
    """The scope's name md_gemm_workspace_size and the earlier
    md_workspace_size give the same sizes."""
    L = md.lib()
    for form in (0, 1, 2):
        for (M, N, K, S) in ((1, 1, 1, 1), (70, 36, 90, 27), (4096, 4096, 4096, 27), (1024, 1024, 1024, 56)):
            a = L.md_gemm_workspace_size(form, M, N, K, S)
            assert a == L.md_workspace_size(form, M, N, K, S) and a > 0


def test_hint_needs_a_certificate_and_a_valid_S():
    """A slice-count hint without a certificate record, a hint that does
    not split into equal bands, and a sign-magnitude hint with another
    digit width are refused before any device work."""
    L = md.lib()
    a, b, c = (ctypes.c_void_p(0x100000 * k) for k in (1, 2, 3))
    cert = ctypes.c_void_p(0x900000)
    for form, hint, beta, with_cert, rc in ((2, 27, 0, False, 7), (2, 37, 0, True, 7), (1, 20, 8, True, 7),
                                            (0, 10, 0, True, 7), (0, 10, 25, True, 7)):
        opts = md.MDOpts()
        opts.form = form
        opts.s_hint = hint
        opts.force_beta = beta
        if with_cert:
            opts.cert = cert
        assert L.md_gemm_ex(2, 0, 0, 4, 4, 4, a, 4, 16, b, 4, 16, c, 4, 16, ctypes.byref(opts), None) == rc
        assert L.md_dot_ex(2, 4, 4, a, 4, 16, b, 4, 16, c, 4, ctypes.byref(opts), None) == rc


def test_binding_refuses_host_buffers():
    """The binding checks a caller's workspace and certificate buffers
    (contiguous, on the operands' device) before calling the library, so a
    host pointer never reaches a kernel.  Without a GPU the operands
    themselves are host tensors: the check on them comes first."""
    import torch
    A = torch.zeros((2, 4, 4), dtype=torch.float64)
    with pytest.raises(ValueError):
        md.gemm_ex(A, A, workspace=torch.zeros(1 << 20, dtype=torch.uint8))
    with pytest.raises(ValueError):
        md._device_buffer(torch.zeros(64, dtype=torch.uint8), "workspace", torch.device("cuda", 0))
    with pytest.raises(ValueError):
        md._device_buffer(torch.zeros((8, 8), dtype=torch.uint8).t(), "cert", torch.device("cpu"))
    opts = md.MDOpts()
    with pytest.raises(ValueError):
        md._slice_opts(opts, torch.device("cuda", 0), 0, 0, 27, None, None)


def test_noalloc_takes_no_workspace():
    """md_gemm_ex_noalloc refuses a caller workspace before any device
    work (its scratch is the library's own array)."""
    L = md.lib()
    a, b, c = (ctypes.c_void_p(0x100000 * k) for k in (1, 2, 3))
    opts = md.MDOpts()
    opts.workspace = ctypes.c_void_p(0x800000)
    opts.workspace_bytes = 1 << 20
    assert L.md_gemm_ex_noalloc(2, 0, 0, 4, 4, 4, a, 4, 16, b, 4, 16, c, 4, 16, ctypes.byref(opts), None) == 7
    assert L.md_gemm_ex_noalloc(3, 0, 0, 4, 4, 4, a, 4, 16, b, 4, 16, c, 4, 16, None, None) == 1
