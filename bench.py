"""Benchmark: quad-double 4096^3 product, INT8-slice vs FP64-slice form.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step is one whole m-double product C = A B (exponent alignment, split,
slice contraction, exact fold, renormalisation) on resident seeded inputs
(leading words U(-1,1), trailing words scaled by 2^-53 U(-1,1)).  The
headline value is the INT8-slice form's effective GFLOP/s, 2 M N K / t, with
balanced 8-bit digits (int8bal); the INT8 form with 7-bit sign-magnitude
digits and the FP64-slice form run beside it with their slice-count rules
and the same 2^-200 target.  Prints one JSON line.

roofline: the dominant kernel is the slice contraction of the headline form;
its algorithmic work per launch is 2 M N K S(S+1)/2 int8 operations (S(S+1)/2
slice multiply-adds per m-double multiply-add), timed with HIP events on the
call's stream around that kernel.

The CPU leg, after all GPU work (skip with --no-cpu), is the only user of
the oracle: cpu_baseline times the exact C oracle on this host's cores over
a bounded sample of output entries, and every "max_log2_err_sampled" field
is the largest error of a grid of sampled GPU outputs against the exact
product (null when the leg is skipped).

ordinary_form: the same product in classical quad-double arithmetic (every
operation renormalised; the paper's comparison baseline), its time, error
and the headline form's speedup over it.

configs (skip with --no-configs): the other workloads of the scope, quad-double
1024^3, double-double 2048^3 and octo-double 1024^3 with the adjoint (three
products per step), hexa-double 1024^3, in the slice forms that apply.

depth_split (skip with --no-split): the benchmark product as exact fixed-point
integers, whole and cut into four depth blocks on the full matrices' exponents,
summed exactly and rounded once; must equal the product's output.

paper_inner_products (skip with --no-dot): the paper's own experiment
(Section 3, Table 2), 1,024 m-double inner products of length 6,144 on its
bit pattern for m = 1, 2, 4, 8, 16, through the batched inner-product entry
point in the three slice forms and with the paper's parameters.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "qd4096"
PEAK_INT8_TOPS = 5000.0      # MI355X dense INT8 matrix peak, TOP/s
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 matrix peak, TFLOP/s


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_tri2d_i8_qd4096_traffic.md")
KERNEL_SOURCES = ("csrc/tri.h", "csrc/trid.h", "csrc/trid.hip", "csrc/slice_common.h", "csrc/renorm.h",
                  "csrc/tri8_s23_28.hip", "build.py")


def kernel_fingerprint():
    """sha256 over the sources of the whole-triangle INT8 kernels, first 16
    hex digits: their headers and unit, the build flags, and of the shared
    internal header only what they take from it (its integer tiling
    constants and the kernel argument block), so that unrelated
    declarations added there keep the stored counter readings valid."""
    import hashlib
    pkg = os.path.join(ROOT, "paper_2606_20863_amd")
    blob = b"".join(open(os.path.join(pkg, f), "rb").read() for f in KERNEL_SOURCES)
    lines = open(os.path.join(pkg, "csrc/mdgemm_internal.h")).read().split("\n")
    keep, inside = [], False
    for ln in lines:
        if ln.startswith("constexpr int ") or ln.startswith("struct GemmArgs"):
            keep.append(ln)
            inside = ln.startswith("struct GemmArgs")
        elif inside:
            keep.append(ln)
            inside = ln != "};"
    blob += "\n".join(keep).encode()
    return hashlib.sha256(blob).hexdigest()[:16]


def int8_kernel_name(info, K):
    """The INT8 slice contraction kernel the library dispatches for these
    parameters (digit width beta = 7 or 8): the whole triangle (S <= 32)
    with two row blocks per wave when the depth is one exactness chunk (for
    balanced S = 27 the variant that shares A through LDS), else one row
    block; two bands over the whole depth for S = 36..64; bands of two row
    blocks per wave otherwise."""
    S, band, b = info["S"], info["band"], info["beta"]
    if band == S and S <= 32:
        if info["kc"] < K:
            return f"k_tri_i8<{S}, false, {b}>"
        # the balanced headline slice count shares A through LDS (trid_shape)
        return "k_tri2d_i8<27, 8, 9>" if (S, b) == (27, 8) else f"k_tri2_i8<{S}, {b}>"
    if 2 * band == S and S % 4 == 0 and 36 <= S <= 64:
        return f"k_duo_i8<{S}, {b}>"
    return f"k_band2_i8<{band}>"


def measured_traffic(kernel: str):
    """HBM bytes per launch of the INT8 slice contraction from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by its reading
    for a plain 1 GiB copy); None when the summary is missing, covers another
    kernel, or the kernel source changed since the counters were taken."""
    path = TRAFFIC_SUMMARY
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", " ", "#")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    want = vals.get("Kernel source fingerprint", "").split("=")[-1].strip()
    if kernel_fingerprint() != want or kernel != vals.get("kernel"):
        return None
    copy = float(vals["copy_bytes"])
    fetch = float(vals["fetch_kib"]) * 1024 * copy / (float(vals["copy_fetch_kib"]) * 1024)
    write = float(vals["write_kib"]) * 1024 * copy / (float(vals["copy_write_kib"]) * 1024)
    return fetch + write


def hip_events(n):
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                        ctypes.c_void_p]
    hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
    evs = []
    for _ in range(n):
        a, b = ctypes.c_void_p(), ctypes.c_void_p()
        assert hip.hipEventCreate(ctypes.byref(a)) == 0
        assert hip.hipEventCreate(ctypes.byref(b)) == 0
        evs.append((a.value, b.value))
    return hip, evs


def elapsed_ms(hip, ev):
    ms = ctypes.c_float()
    rc = hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(ev[0]), ctypes.c_void_p(ev[1]))
    assert rc == 0, rc
    return float(ms.value)


def progress(msg):
    """One line per finished phase on stderr (the JSON line goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_form(md, torch, A, B, form, steps, warmup):
    hip, evs = hip_events(steps)
    for _ in range(warmup):
        C, info = md.gemm_ex(A, B, form=form)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        C, info = md.gemm_ex(A, B, form=form, events=evs[i])
    info["rule"] = "rho" if info["G"] != info["G_span"] or info["G_rho"] >= 0 else "span"
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = [elapsed_ms(hip, e) for e in evs]
    for a, b in evs:
        hip.hipEventDestroy(ctypes.c_void_p(a))
        hip.hipEventDestroy(ctypes.c_void_p(b))
    ms = (t1 - t0) * 1e3 / steps
    return C, info, ms, sum(kern) / len(kern)


# Sampled outputs of the GPU runs, kept for the CPU leg: the oracle runs
# only there, after all GPU work (with --no-cpu the error fields stay null).
_ERROR_CHECKS = []


def defer_error(target, key, A, B, C, n=8):
    """Keep an n x n grid of outputs of C = A B (numpy or device planes)
    with the rows of A and the columns of B they need; the CPU leg writes
    max log2(|C - C*| / (|A||B|)) over them into target[key]."""
    import numpy as np
    M, N = C.shape[1], C.shape[2]
    ri = np.linspace(0, M - 1, n).astype(np.int64)
    ci = np.linspace(0, N - 1, n).astype(np.int64)
    ii = np.arange(n, dtype=np.int64).repeat(n)
    jj = np.tile(np.arange(n, dtype=np.int64), n)
    if hasattr(C, "cpu"):
        import torch
        Cq = C[:, torch.from_numpy(ri[ii]).to(C.device), torch.from_numpy(ci[jj]).to(C.device)].cpu().numpy()
    else:
        Cq = C[:, ri[ii], ci[jj]]
    defer_entries(target, key, np.ascontiguousarray(A[:, ri, :]), np.ascontiguousarray(B[:, :, ci]),
                  ii, jj, np.ascontiguousarray(Cq.T))


def defer_entries(target, key, A, B, ii, jj, Cq):
    """Entries (ii[q], jj[q]) of A B computed as Cq[q] (m words), checked
    by the CPU leg."""
    target[key] = None
    _ERROR_CHECKS.append((target, key, A, B, ii, jj, Cq))


def resolve_errors():
    """The CPU leg's error check of every deferred sample (exact C oracle)."""
    import numpy as np
    from oracle import coracle
    for target, key, A, B, ii, jj, Cq in _ERROR_CHECKS:
        _, absab, err = coracle.exact_entries(A, B, ii, jj, Cq)
        rel = np.abs(err) / absab
        target[key] = round(float(np.log2(max(rel.max(), 2.0 ** -1074))), 2)
    _ERROR_CHECKS.clear()


# Table 2 of the paper: one CPU core, 1,024 inner products of length 6,144,
# milliseconds ("vectorized" is the error-free method, "ordinary" classical
# m-double arithmetic).  Context only: other hardware, other parameters.
PAPER_TABLE2_MS = {1: (12, 30), 2: (158, 69), 4: (1977, 318), 8: (6428, 1520), 16: (40780, 9491)}


def paper_inner_products(md, torch, steps=5):
    """The paper's experiment on the GPU: 1,024 inner products of length
    6,144 on the bit pattern, m = 1, 2, 4, 8, 16, through md_dot_ex in the
    two INT8 forms and the FP64 form (the library's slice rule) and with the
    paper's own parameters (FP64 form, beta = 13, S = 4m).  Whole-call
    milliseconds (inputs resident), the contraction and fold alone from HIP
    events, and the largest error over 8 sampled pairs against the exact
    products (checked by the CPU leg) relative to sum |x||y|.  The balanced
    INT8 form also on the rule's S as a hint (no host round trip), with the
    HBM bytes a call must read (the m words of both operands, 2 8 m batch n)
    and that rate against 8 TB/s.  Beside them, for every m: the same
    products in ordinary m-double arithmetic on the GPU (md_dot_ordinary),
    and the ordinary-to-error-free time ratio beside the paper's one-core
    ratio from Table 2."""
    import numpy as np
    import mdinputs
    X16, Y16 = mdinputs.paper_dot_workload(16)
    hip, _ = hip_events(1)
    pairs = np.linspace(0, X16.shape[1] - 1, 8).astype(np.int64)
    idx = np.arange(len(pairs), dtype=np.int64)
    rows = {}
    for m in mdinputs.PAPER_DOT["m"]:
        X = torch.from_numpy(np.ascontiguousarray(X16[:m])).cuda()
        Y = torch.from_numpy(np.ascontiguousarray(Y16[:m])).cuda()
        Xs = np.ascontiguousarray(X16[:m, pairs, :])
        Ys = np.ascontiguousarray(np.transpose(Y16[:m, pairs, :], (0, 2, 1)))
        row = {"paper_cpu_ms_ordinary": PAPER_TABLE2_MS[m][0],
               "paper_cpu_ms_vectorized": PAPER_TABLE2_MS[m][1]}
        for label, kw in (("int8bal", dict(form="int8bal")), ("int8", dict(form="int8")),
                          ("fp64", dict(form="fp64")),
                          ("fp64_paper_params", dict(form="fp64", force_S=4 * m, force_beta=13))):
            for _ in range(2):
                md.dot_ex(X, Y, **kw)
            torch.cuda.synchronize()
            _, evs = hip_events(steps)
            t0 = time.perf_counter()
            for e in evs:
                out, info = md.dot_ex(X, Y, events=e, **kw)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            kern = sum(elapsed_ms(hip, e) for e in evs) / steps
            for a, b in evs:
                hip.hipEventDestroy(ctypes.c_void_p(a))
                hip.hipEventDestroy(ctypes.c_void_p(b))
            Cq = np.ascontiguousarray(out.cpu().numpy()[:, pairs].T)
            row[label] = {"S": info["S"], "beta": info["beta"], "ms_per_call": round(ms, 4),
                          "contraction_fold_ms": round(kern, 4)}
            defer_entries(row[label], "max_log2_err_sampled", Xs, Ys, idx, idx, Cq)
            if label == "int8bal":
                cert = md.new_cert()
                hint = dict(form="int8bal", s_hint=info["S"], cert=cert)
                oh, _ = md.dot_ex(X, Y, **hint)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    oh, _ = md.dot_ex(X, Y, **hint)
                torch.cuda.synchronize()
                msh = (time.perf_counter() - t0) * 1e3 / steps
                nbytes = 2 * 8 * m * X.shape[1] * X.shape[2]
                row[label].update({"ms_per_call_hint": round(msh, 4),
                                   "hint_equals_rule": bool(torch.equal(oh, out)),
                                   "hint_certificate_flags": md.read_cert(cert)["flags"],
                                   "input_bytes_per_call": nbytes,
                                   "hint_hbm_frac": round(nbytes / (msh * 1e-3) / 8e12, 4)})
        md.dot_ordinary(X, Y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            oo = md.dot_ordinary(X, Y)
        torch.cuda.synchronize()
        mso = (time.perf_counter() - t0) * 1e3 / steps
        row["ordinary"] = {"arithmetic": "ordinary m-double, every operation renormalised "
                                         "(md_dot_ordinary, 64 partial sums per pair)",
                           "ms_per_call": round(mso, 4)}
        defer_entries(row["ordinary"], "max_log2_err_sampled", Xs, Ys, idx, idx,
                      np.ascontiguousarray(oo.cpu().numpy()[:, pairs].T))
        row["gpu_ordinary_over_int8bal"] = round(mso / row["int8bal"]["ms_per_call"], 3)
        row["gpu_ordinary_over_int8bal_hint"] = round(mso / row["int8bal"]["ms_per_call_hint"], 3)
        row["paper_cpu_ordinary_over_vectorized"] = round(PAPER_TABLE2_MS[m][0] / PAPER_TABLE2_MS[m][1], 3)
        rows[f"m{m}"] = row
        progress(f"inner products m={m} done")
        del X, Y
    return {"workload": "1024 inner products of length 6144, the paper's bit pattern (Section 2), "
                        "m-double inputs, one md_dot_ex call each",
            "target_bits": "50 m", "results": rows}


def other_configs(md, torch, steps=3, only=None):
    """The scope's other workloads, each timed as whole steps (inputs
    resident; per form one warm-up step, then at least ``steps`` steps and
    about 20 ms of them, at most 50): double-double 64^3 (per-call microseconds, eager and as a
    HIP graph replay); quad-double 1024^3 forward; double-double 2048^3 and
    octo-double 1024^3 forward + adjoint (C = A B, dA = W B^T, dB = A^T W:
    three products per step); hexa-double 1024^3 forward (leading words
    2^U(-6,6), seed 16).  Per form: milliseconds per step, effective GFLOP/s
    (2 M N K per product), the slice contractions with their folds from HIP
    events, their fraction of the matrix-core peak (algorithmic work
    2 M N K S(S+1)/2 per product), and the largest error of 64 sampled
    entries against the exact product (checked by the CPU leg), of the
    forward product and, with the adjoint, of both gradients."""
    import numpy as np
    import mdinputs
    hip, _ = hip_events(1)
    r16 = np.random.Generator(np.random.PCG64(16))
    cases = [
        ("qd1024", "quad-double 1024^3, forward", lambda: mdinputs.workload("qd1024", with_w=True),
         False, ("int8bal", "int8", "fp64")),
        ("dd2048", "double-double 2048^3, forward + adjoint", lambda: mdinputs.workload("dd2048", with_w=True),
         True, ("fp64", "int8bal")),
        ("od1024", "octo-double 1024^3, forward + adjoint", lambda: mdinputs.workload("od1024", with_w=True),
         True, ("int8bal", "int8", "fp64")),
        ("hd1024", "hexa-double 1024^3 (leading words 2^U(-6,6)), forward",
         lambda: (mdinputs.mdouble(r16, 16, (1024, 1024), ("log2uniform", 6.0)),
                  mdinputs.mdouble(r16, 16, (1024, 1024), ("log2uniform", 6.0)), None),
         False, ("int8bal", "int8", "fp64")),
    ]
    res = {}
    if only is None or "dd64" in only:
        res["dd64"] = small_case(md, torch)
        progress("workload dd64 done")
    for name, label, make, adjoint, forms in cases:
        if only is not None and name not in only:
            continue
        Ah, Bh, Wh = make()
        A = torch.from_numpy(Ah).cuda()
        B = torch.from_numpy(Bh).cuda()
        W = torch.from_numpy(Wh).cuda() if adjoint else None
        calls = [dict(A=A, B=B)]
        if adjoint:
            calls += [dict(A=W, B=B, transB=True), dict(A=A, B=W, transA=True)]
        m, M, K = Ah.shape
        N = Bh.shape[2]
        flop = 2.0 * M * N * K * len(calls)
        row = {"label": label, "m": m}
        for form in forms:
            for c in calls:
                C, _ = md.gemm_ex(c["A"], c["B"], transA=c.get("transA", False),
                                  transB=c.get("transB", False), form=form)
            torch.cuda.synchronize()
            # at least `steps` steps and about 20 ms of them, at most 50 (the
            # slice rule's read-back keeps the host in step with the device)
            _, evs = hip_events(50 * len(calls))
            t0 = time.perf_counter()
            infos = []
            nst = 0
            while nst < 50 and (nst < steps or time.perf_counter() - t0 < 0.02):
                st = nst
                nst += 1
                for q, c in enumerate(calls):
                    Cq, info = md.gemm_ex(c["A"], c["B"], transA=c.get("transA", False),
                                          transB=c.get("transB", False), form=form,
                                          events=evs[st * len(calls) + q])
                    if q == 0:
                        C = Cq
                    elif q == 1:
                        dA = Cq
                    else:
                        dB = Cq
                    infos.append(info)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / nst
            kern = sum(elapsed_ms(hip, e) for e in evs[:nst * len(calls)]) / nst
            for a, b in evs:
                hip.hipEventDestroy(ctypes.c_void_p(a))
                hip.hipEventDestroy(ctypes.c_void_p(b))
            ops = sum(2.0 * M * N * K * i["S"] * (i["S"] + 1) / 2 for i in infos[:len(calls)])
            peak = PEAK_FP64_TFLOPS if form == "fp64" else PEAK_INT8_TOPS
            row[form] = {"S": [i["S"] for i in infos[:len(calls)]], "beta": infos[0]["beta"],
                         "steps": nst, "ms_per_step": round(ms, 4),
                         "effective_gflops": round(flop / (ms * 1e-3) / 1e9, 2),
                         "contraction_fold_ms": round(kern, 4),
                         "frac_peak": round(ops / (kern * 1e-3) / 1e12 / peak, 4)}
            defer_error(row[form], "max_log2_err_sampled", Ah, Bh, C)
            if adjoint:
                # the gradients: dA = W B^T and dB = A^T W on 8 x 8 grids each
                defer_error(row[form], "max_log2_err_dA_sampled", Wh,
                            np.ascontiguousarray(np.transpose(Bh, (0, 2, 1))), dA)
                defer_error(row[form], "max_log2_err_dB_sampled",
                            np.ascontiguousarray(np.transpose(Ah, (0, 2, 1))), Wh, dB)
        res[name] = row
        progress(f"workload {name} done")
        del A, B, W, calls, C
        if adjoint:
            del dA, dB
        torch.cuda.empty_cache()
    return res


def depth_split(md, torch, A, B, C, info, blocks=4, steps=2):
    """The benchmark product as exact fixed-point integers: the whole
    product's integer (md_gemm_fixed), and the depth cut into equal blocks
    split on the full matrices' exponents (md_exponents), their integers
    summed (md_fixed_add) and rounded once (md_fixed_round) -- one GPU's
    share of a depth-split product and its exact reduction; the blocks
    report refused exponents into a device word, so nothing waits.  Milliseconds
    per step of each, and whether the rounded sum equals C (md_gemm_ex's
    output for the same S) in every entry."""
    form = "int8bal" if info["beta"] == 8 else ("int8" if info["beta"] == 7 else "fp64")
    S, beta = info["S"], info["beta"]
    m, M, K = A.shape
    N = B.shape[2]
    nlimb = md.fixed_limbs(beta, S, K)
    cuts = [K * q // blocks for q in range(blocks + 1)]

    def whole():
        return md.gemm_fixed(A, B, S=S, beta=beta, form=form)[:2]

    flags = torch.zeros(1, dtype=torch.int32, device=A.device)

    def split():
        E, F = md.exponents(A, B)
        acc = sc = None
        for a, b in zip(cuts[:-1], cuts[1:]):
            Xb, sc, _ = md.gemm_fixed(A[:, :, a:b], B[:, a:b, :], E, F, S=S, beta=beta, form=form,
                                      nlimb=nlimb, flags=flags)
            acc = Xb if acc is None else md.fixed_add(acc, Xb, out=acc)
        return md.fixed_round(acc, sc, m)

    res = {"form": form, "S": S, "beta": beta, "limbs": nlimb, "blocks": blocks}
    for name, fn in (("whole_fixed_ms", whole), ("split_sum_round_ms", split)):
        out = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = fn()
        torch.cuda.synchronize()
        res[name] = round((time.perf_counter() - t0) * 1e3 / steps, 3)
        if name == "split_sum_round_ms":
            res["rounded_sum_equals_product"] = bool(torch.equal(out, C))
            res["exponents_all_taken"] = int(flags.item()) == 0
        del out
        torch.cuda.empty_cache()
    return res


def small_case(md, torch, reps=200):
    """Double-double 64^3, the smallest workload, where launches and the
    host round trip dominate: microseconds per product (a) eager with the
    slice rule (one host synchronisation for the exponent spans), (b) eager
    with the rule's S as a hint and a caller workspace (the certificate
    checked on the device, no synchronisation; its record must carry no
    flag), (c) eager with the rule's S forced and a caller workspace (kernel
    launches only), (d) replays of a HIP graph holding (c), whose output
    must equal (a)'s."""
    import mdinputs
    Ah, Bh = mdinputs.workload("dd64")
    A = torch.from_numpy(Ah).cuda()
    B = torch.from_numpy(Bh).cuda()
    m, M, K = Ah.shape
    N = Bh.shape[2]
    row = {"label": "double-double 64^3 (launch-bound)", "m": m}

    def per_call_us(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return round((time.perf_counter() - t0) * 1e6 / reps, 2)

    for form in ("fp64", "int8bal", "int8"):
        C, info = md.gemm_ex(A, B, form=form)
        kw = dict(form=form, force_S=info["S"], force_beta=info["beta"])
        ws = torch.empty(md.lib().md_gemm_workspace_size(md._FORMS[form], M, N, K, info["S"]),
                         dtype=torch.uint8, device="cuda")
        Cg = torch.empty_like(C)
        us_rule = per_call_us(lambda: md.gemm_ex(A, B, C, form=form))
        cert = md.new_cert()
        Ch = torch.empty_like(C)
        hint = dict(form=form, s_hint=info["S"], force_beta=info["beta"] if form == "fp64" else 0, cert=cert)
        us_hint = per_call_us(lambda: md.gemm_ex(A, B, Ch, workspace=ws, **hint))
        c = md.read_cert(cert)
        us_forced = per_call_us(lambda: md.gemm_ex(A, B, C, workspace=ws, **kw))
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            md.gemm_ex(A, B, Cg, workspace=ws, **kw)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            md.gemm_ex(A, B, Cg, workspace=ws, **kw)
        Cg.zero_()
        us_graph = per_call_us(g.replay)
        row[form] = {"S": info["S"], "beta": info["beta"], "eager_rule_us": us_rule,
                     "eager_hint_us": us_hint, "hint_certificate_flags": c["flags"],
                     "hint_equals_rule": bool(torch.equal(Ch, C)),
                     "eager_forced_us": us_forced, "graph_replay_us": us_graph,
                     "graph_equals_eager": bool(torch.equal(Cg, C))}
        defer_error(row[form], "max_log2_err_sampled", Ah, Bh, C)
        del g
    return row


def host_cpu():
    """The host's CPU model, physical cores and logical CPUs (from
    /proc/cpuinfo), and the CPUs this process may run on."""
    model, cores, logical = None, set(), 0
    try:
        phys = core = None
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key, val = key.strip(), val.strip()
                if key == "processor":
                    logical += 1
                elif key == "model name" and model is None:
                    model = val
                elif key == "physical id":
                    phys = val
                elif key == "core id":
                    core = val
                    cores.add((phys, core))
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count()
    return {"cpu_model": model, "physical_cores": len(cores) or None, "logical_cpus": logical or os.cpu_count(),
            "cpus_allowed": allowed}


def cpu_baseline(A, B, K):
    """The exact C oracle on whole output rows of the same product."""
    import numpy as np
    from oracle import coracle
    N = B.shape[2]
    rows = 32
    ii = np.arange(rows, dtype=np.int64).repeat(N)
    jj = np.tile(np.arange(N, dtype=np.int64), rows)
    t0 = time.perf_counter()
    coracle.exact_entries(A, B, ii, jj)
    dt = time.perf_counter() - t0
    gflops = 2.0 * K * ii.shape[0] / dt / 1e9
    return {"value": round(gflops, 6), "unit": "GFLOP/s", "cores": coracle.threads(),
            "kind": "oracle", **host_cpu(),
            "sample": f"{rows} full rows x {N} columns of the {WORKLOAD} product "
                      f"(exact superaccumulator oracle, {dt:.1f} s); rate scaled per output entry"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--sm-steps", type=int, default=3,
                    help="timed calls of the sign-magnitude INT8 form (7-bit digits)")
    ap.add_argument("--ordinary-steps", type=int, default=1,
                    help="timed calls of the ordinary quad-double product (0 skips it)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-dot", action="store_true",
                    help="skip the paper's inner-product workload (m = 1..16)")
    ap.add_argument("--no-split", action="store_true",
                    help="skip the fixed-point depth split of the benchmark product")
    ap.add_argument("--configs", default="",
                    help="comma-separated subset of the other workloads (dd64, qd1024, dd2048, od1024, hd1024)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (qd1024, dd2048 and od1024 with the adjoint, hd1024)")
    ap.add_argument("--forms", default="int8bal,int8,fp64",
                    help="slice forms to run (int8bal, the balanced 8-bit digits, is the "
                         "headline; the sign-magnitude int8 and the fp64 forms run beside it)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="before the timed region, copy 1 GiB device to device once: a plain "
                         "kernel of known traffic for scaling hardware byte counters")
    args = ap.parse_args()
    forms = set(args.forms.split(","))
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import mdinputs
    import paper_2606_20863_amd as md

    Ah, Bh = mdinputs.workload(WORKLOAD)
    m, M, K = Ah.shape
    N = Bh.shape[2]
    A = torch.from_numpy(Ah).cuda()
    B = torch.from_numpy(Bh).cuda()
    torch.cuda.synchronize()
    if args.calibrate_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    head = "int8bal" if "int8bal" in forms else "int8"
    progress(f"{WORKLOAD} inputs resident")
    C8, info8, ms8, kern8 = run_form(md, torch, A, B, head, args.steps, args.warmup)
    progress(f"{head} form: {ms8:.3f} ms per call")
    if "fp64" not in forms:
        out = {"metric": f"QD-GEMM 4096^3 effective GFLOP/s ({head} form only)",
               "ms_per_call": round(ms8, 4), "gemm_kernel_ms": round(kern8, 4), "S": info8["S"],
               "kernel": int8_kernel_name(info8, K)}
        if args.configs:
            # profiling runs of chosen workloads beside the one headline form
            del A, B, C8
            torch.cuda.empty_cache()
            out["configs"] = other_configs(md, torch, only=args.configs.split(","))
        print(json.dumps(out))
        return
    sm = None
    if head == "int8bal" and "int8" in forms and args.sm_steps > 0:
        Csm, infosm, mssm, kernsm = run_form(md, torch, A, B, "int8", args.sm_steps, 1)
        sm = (Csm.cpu().numpy(), infosm, mssm, kernsm)
        del Csm
    C64, info64, ms64, kern64 = run_form(md, torch, A, B, "fp64", args.fp64_steps, 1)
    progress(f"fp64 form: {ms64:.3f} ms per call")

    # the ordinary (classical) quad-double product on the same inputs, the
    # paper's comparison baseline; one warm-up and args.ordinary_steps timed
    ord_ms = None
    if args.ordinary_steps > 0:
        Co = md.gemm_ordinary(A, B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.ordinary_steps):
            Co = md.gemm_ordinary(A, B)
        torch.cuda.synchronize()
        ord_ms = (time.perf_counter() - t0) * 1e3 / args.ordinary_steps
        Coh = Co.cpu().numpy()
        del Co
        progress(f"ordinary form: {ord_ms:.1f} ms per call")

    flop = 2.0 * M * N * K
    eff8 = flop / (ms8 * 1e-3) / 1e9
    eff64 = flop / (ms64 * 1e-3) / 1e9
    S8, S64 = info8["S"], info64["S"]
    ops8 = flop * S8 * (S8 + 1) / 2
    ops64 = flop * S64 * (S64 + 1) / 2
    ach8 = ops8 / (kern8 * 1e-3) / 1e12
    ach64 = ops64 / (kern64 * 1e-3) / 1e12

    kname8 = int8_kernel_name(info8, K)
    traffic8 = measured_traffic(kname8)
    traffic8 = None if traffic8 is None else int(traffic8)

    def int8_summary(info, ms, kern, steps):
        S = info["S"]
        ops = flop * S * (S + 1) / 2
        return {"S": S, "beta": info["beta"], "kc": info["kc"], "band": info["band"],
                "steps": steps, "ms_per_call": round(ms, 4), "gemm_kernel_ms": round(kern, 4),
                "kernel": int8_kernel_name(info, K),
                "effective_gflops": round(flop / (ms * 1e-3) / 1e9, 3),
                "mfma_int8_tops": round(ops / (kern * 1e-3) / 1e12, 3),
                "max_log2_err_sampled": None,
                "certified_log2_bound": round(info["log2_bound"], 2)}

    head_form = int8_summary(info8, ms8, kern8, args.steps)
    head_form["digits"] = ("balanced 8-bit digits in [-128, 127] on the grid 2^(E+2)" if head == "int8bal"
                           else "7-bit sign-magnitude digits")
    out = {
        "metric": "QD-GEMM 4096^3 effective GFLOP/s: INT8-slice vs FP64-slice MFMA, same error",
        "value": round(eff8, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms8, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD}: quad-double (m=4) C = A B, M=N=K=4096, leading words "
                               "U(-1,1), trailing words 2^-53 U(-1,1)",
                   "M": M, "N": N, "K": K, "m": m, "target_bits": info8["target_bits"],
                   "s_rule": info8.get("rule", "rho")},
        "headline_form": head,
        f"{head}_form": head_form,
        "fp64_form": {"S": S64, "beta": info64["beta"], "kc": info64["kc"], "band": info64["band"],
                      "steps": args.fp64_steps, "ms_per_call": round(ms64, 4),
                      "gemm_kernel_ms": round(kern64, 4), "effective_gflops": round(eff64, 3),
                      "mfma_tflops": round(ach64, 3), "frac_fp64_peak": round(ach64 / PEAK_FP64_TFLOPS, 4),
                      "max_log2_err_sampled": None,
                      "certified_log2_bound": round(info64["log2_bound"], 2)},
        "int8_over_fp64": round(eff8 / eff64, 3),
        "int8_sign_magnitude_form": None if sm is None else dict(
            int8_summary(sm[1], sm[2], sm[3], args.sm_steps),
            digits="7-bit sign-magnitude digits (the paper's bit-field cut)",
            headline_speedup=round(sm[2] / ms8, 3)),
        "ordinary_form": None if ord_ms is None else {
            "arithmetic": "classical quad-double, every multiply and add renormalised (md_gemm_ordinary)",
            "steps": args.ordinary_steps, "ms_per_call": round(ord_ms, 3),
            "effective_gflops": round(flop / (ord_ms * 1e-3) / 1e9, 3),
            "max_log2_err_sampled": None,
            "headline_form_speedup": round(ord_ms / ms8, 2)},
        "roofline": {"bound": "mfma", "kernel": kname8,
                     "achieved": round(ach8, 3), "peak": PEAK_INT8_TOPS, "unit": "TFLOP/s",
                     "frac": round(ach8 / PEAK_INT8_TOPS, 4), "traffic": traffic8,
                     "work_per_launch": f"2*M*N*K*S(S+1)/2 = {ops8:.4e} int8 ops (unit: int8 TOP/s)",
                     "algorithmic_bytes_per_launch": int(2 * S8 * M * K + 8 * m * M * N)},
    }
    if not args.no_split:
        out["depth_split"] = depth_split(md, torch, A, B, C8, info8)
        progress("depth split done")
    defer_error(head_form, "max_log2_err_sampled", Ah, Bh, C8, n=64)
    head_form["error_sample"] = "64 x 64 grid of entries (4,096), exact C oracle"
    defer_error(out["fp64_form"], "max_log2_err_sampled", Ah, Bh, C64)
    if sm is not None:
        defer_error(out["int8_sign_magnitude_form"], "max_log2_err_sampled", Ah, Bh, sm[0])
    if ord_ms is not None:
        defer_error(out["ordinary_form"], "max_log2_err_sampled", Ah, Bh, Coh)
    if not args.no_dot:
        del A, B, C8, C64
        torch.cuda.empty_cache()
        out["paper_inner_products"] = paper_inner_products(md, torch)
    if not args.no_configs:
        if args.no_dot:
            del A, B, C8, C64
            torch.cuda.empty_cache()
        out["configs"] = other_configs(md, torch, only=args.configs.split(",") if args.configs else None)
    # the CPU leg: every use of the oracle, after all GPU work
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(Ah, Bh, K)
        progress("cpu baseline timed")
        resolve_errors()
        progress("sampled errors checked")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
