"""Benchmark of the Gray-code permanent on one MI355X.

Default workload: the 40 x 40 top-left block of a 1600-mode Haar unitary
(complex128, seed 20190402), its whole permanent in FP64 with double-double
sums (2^39 Gray terms).  A step is one full library call: staging, the walk
over all 2^(n-1) terms, the fixed-order reduction and the result on the host;
the matrix is resident in HBM before the timed region starts.  The metric
counts n * 2^(n-1) element-steps per permanent.

Printed: one JSON line with the throughput, the roofline of the walk kernel
(VALU lane-operations of the algorithm per second against the chip's vector
issue peak; the kernel's own duration comes from HIP events recorded by the
library on the launch stream), the CPU oracle timed on the host cores, the
GPU against the oracle's own sample, and -- outside the timed region -- the
same permanent with plain FP64 sums and with FP32 products (their relative
difference to the timed result), and the batched distribution study (100000
Haar blocks, n uniform on 8..24) as permanents/s.

Other workloads (--workload c1|c2|c4|c5|c6|c7|c8|c9) are for manual runs: c1
the 20 x 20 complex call; c2 the exact 30 x 30 0/1 permanent; c4 the
batched study alone; c5 (48x48 real, 2^47 terms, minutes per permanent) runs
as 16 perm_partial slices with a progress line each; c6 is the
repeated-column path (Eq. ryser2) on a 48-photon output with two photons in
each of 24 modes; c7 is the band transfer matrix (App. C) on a batch of
64 x 64 band matrices; c8 the exact sparse path (App. B) on the paper's
identity + Bernoulli(p) matrices; c9 the random-ensemble study (Sec. III) on
100000 Ginibre 20 x 20 matrices.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from types import SimpleNamespace

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 VALU lanes x 2.4 GHz = 3.93e13 lane-operations/s (FP64 add,
# mul and fma each take one slot; 78.6 TFLOP/s counts an fma as two flops).
PEAK_LANE_OPS = 256 * 64 * 2.4e9

SEED_C2 = 20190413


def algorithmic_ops_per_term(kind: str, n: int, col0_nonzeros: int = 0,
                             walk_variant: int = 0) -> float:
    """VALU lane-operations the method needs per Gray term (App. A, subpermanent):
    n row-sum updates, n-1 multiplies, 1 signed accumulate (complex: 2n updates,
    n-1 complex multiplies of 4 ops, 2 accumulates).

    The pair-shared 0/1 walk evaluates the two terms of a pair as S (D1 - D0):
    per pair m + n updates (m = ones in the flipped column), n - M - 1 static
    multiplies (M = n // 3), 2 (M - 1) dynamic ones, one subtraction, one
    multiply by S and one accumulate: 2n + m + M per pair.

    The banded walk (walk_variant 2) takes two pairs as S' E (D1 - D0) each,
    S' shared (E = (n - M) // 2 rows): per quad n + M + E + 2m updates,
    n - M - E - 1 shared multiplies, and per pair E - 1 + 2 (M - 1) dynamic
    ones, one subtraction, two multiplies by S' and E and one accumulate:
    2n + 4M + 2E + 2m + 1 per quad."""
    if kind == "complex":
        return 2 * n + 4 * (n - 1) + 2
    if col0_nonzeros and walk_variant == 2:
        M = n // 3
        E = (n - M) // 2
        return (2 * n + 4 * M + 2 * E + 2 * col0_nonzeros + 1) / 4.0
    if col0_nonzeros:
        return (2 * n + col0_nonzeros + n // 3) / 2.0
    return 2 * n


KERNEL_SOURCES = {
    "int01": ["kern_int01.hip", "perm_exact.hpp"],
    "real": ["kern_real.hip", "perm_walk.hpp"],
    "complex": ["kern_complex.hip", "perm_walk.hpp"],
    "band": ["kern_band.hip"],
    "mixed": ["kern_mixed.hip", "perm_exact.hpp", "perm_walk.hpp", "perm_cases_lo.inc",
              "perm_cases_hi.inc"],
    "batched": ["kern_batched.hip", "perm_walk.hpp"],
}


def _strip_comments(src: str) -> str:
    """C/C++ source without its comments and blank lines (the kernel sources
    hold no string literal containing comment markers)."""
    import re
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(line.rstrip() for line in src.splitlines() if line.strip())


def source_sha(kind):
    """Hash of the code (comments excluded) that a kernel is built from: a
    counter summary stays valid across comment edits, not code edits."""
    import hashlib
    base = os.path.join(ROOT, "paper_1904_06229_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind] + ["perm_device.hpp", "perm_internal.hpp"]:
        with open(os.path.join(base, f), encoding="utf-8") as fh:
            h.update(_strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def parse_traffic_line(line):
    """The key=value fields of a TRAFFIC line; a kernel name may hold spaces
    ("band_kernel<5, true>")."""
    import re
    return dict(re.findall(r"(\w+)=(.*?)(?=\s+\w+=|\s*$)", line[len("TRAFFIC "):]))


def profiled_traffic(kernel, kind):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size), or None
    when there is none or the kernel's source changed since it was taken."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    want = source_sha(kind)
    for fn in sorted(os.listdir(pdir)):
        with open(os.path.join(pdir, fn)) as fh:
            for line in fh:
                if not line.startswith("TRAFFIC "):
                    continue
                kv = parse_traffic_line(line)
                if kv.get("kernel") == kernel and kv.get("src") == want:
                    return int(kv["fetch_bytes"]) + int(kv["write_bytes"])
    return None


def calibrate_copy():
    """Two plain 256 MiB device copies, whose FETCH_SIZE and WRITE_SIZE under
    rocprofv3 give the scale of those counters for the kernels measured in
    the same run."""
    import torch
    src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")  # 256 MiB
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=None,
                   help="timed steps (default 20; c3, c4, c8: 5, 3, 3; c6: 10; 1 for a whole "
                        "sliced permanent)")
    p.add_argument("--warmup", type=int, default=None,
                   help="untimed steps first (default 3; c3, c4, c6, c8: 1; 0 for a whole "
                        "sliced permanent)")
    p.add_argument("--workload", default="c3",
                   choices=["c1", "c2", "c3", "c4", "c5", "c6", "c7", "c8", "c9", "dense"])
    p.add_argument("--n", type=int, default=48,
                   help="dense: matrix size (2..64); c6: even size (4..64), n/2 columns x 2")
    p.add_argument("--kind", default="complex", choices=["complex", "real"],
                   help="dense: complex Ginibre/sqrt(n) or real N(0,1) entries")
    p.add_argument("--count", type=int, default=100000, help="c4: number of matrices")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-autotune", action="store_true",
                   help="c4: use the default chunk lengths instead of tuning them first")
    p.add_argument("--blocks", type=int, default=0)
    p.add_argument("--log2-chunk", type=int, default=0)
    p.add_argument("--precision", default="dd")
    p.add_argument("--slices", type=int, default=0,
                   help="evaluate each permanent as this many perm_partial slices, a progress "
                        "line per slice (c5 uses 16 unless given)")
    p.add_argument("--checkpoint", default=None, help="slice checkpoint file (resume)")
    p.add_argument("--terms-log2", type=int, default=0,
                   help="time only the first 2^K Gray terms (perm_partial); labelled as a prefix")
    p.add_argument("--no-batched", action="store_true",
                   help="c3: leave out the batched study that follows the timed region")
    p.add_argument("--no-compare", action="store_true",
                   help="c1, c3: leave out the plain-FP64 and FP32-product runs after the timed "
                        "region")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="also run a plain 256 MiB device copy (scale reference for HBM counters)")
    args = p.parse_args()
    # A whole 48 x 48 permanent (minutes) is one step by default; a checkpoint
    # resumes one permanent, so it allows exactly one step and no warmup.
    sliced = bool(args.slices or args.checkpoint or
                  (args.workload == "c5" and not args.terms_log2))
    if args.checkpoint and ((args.steps or 1) != 1 or (args.warmup or 0) != 0):
        p.error("--checkpoint resumes one permanent: it takes --steps 1 --warmup 0")
    # defaults keep the timed work of a manual run near a minute or less
    steps, warmup = {"c3": (5, 1), "c4": (3, 1), "c6": (10, 1), "c8": (3, 1), "c9": (5, 1)}.get(
        args.workload, (20, 3))
    if sliced:
        steps, warmup = 1, 0
    if args.steps is None:
        args.steps = steps
    if args.warmup is None:
        args.warmup = warmup
    if args.steps < 1 or args.warmup < 0:
        p.error("--steps must be >= 1 and --warmup >= 0")
    if args.workload == "dense" and not 2 <= args.n <= 64:
        p.error("--n must be in 2..64")
    if args.workload == "c6" and (args.n % 2 or not 4 <= args.n <= 64):
        p.error("c6: --n must be even, in 4..64")
    return args


def make_workload(name, args=None):
    from paper_1904_06229_amd import inputs
    if name == "dense":
        n, seed = args.n, 20190400 + args.n
        if args.kind == "complex":
            return "complex", n, inputs.complex_gaussian(n, seed, scale=n ** -0.5), \
                f"{n}x{n} complex128 Ginibre/sqrt(n), seed {seed}"
        return "real", n, inputs.real_gaussian(n, seed), f"{n}x{n} real N(0,1), seed {seed}"
    if name == "c1":
        n = 20
        return "complex", n, inputs.complex_gaussian(n, 20190401, scale=n ** -0.5), \
            "20x20 complex128 Ginibre/sqrt(n), seed 20190401"
    if name == "c2":
        n = 30
        return "int01", n, inputs.bernoulli01(n, SEED_C2), \
            f"30x30 0/1 Bernoulli(1/2), seed {SEED_C2}, exact (int128)"
    if name == "c3":
        n = 40
        return "complex", n, inputs.haar_block(n, n * n, 20190402), \
            "40x40 top-left block of a 1600-mode Haar unitary, seed 20190402"
    if name == "c5":
        n = 48
        return "real", n, inputs.real_gaussian(n, 20190403), "48x48 real N(0,1), seed 20190403"
    raise ValueError(name)


def cpu_baseline(kind, n, A):
    """The oracle, as it stands, on a bounded sample of the same workload.
    Returns the bench-line record, the sample's size and the oracle's value
    over it."""
    import oracle
    oracle.build(force=False)
    threads = oracle.default_threads()
    if kind == "int01":
        # Ryser over a prefix of the 2^n subsets, sized to ~10-20 s on the host.
        count = 1 << n if n <= 30 else 1 << 30
        t0 = time.perf_counter()
        got = oracle.ryser_range(A, 0, count, threads=threads)
        dt = time.perf_counter() - t0
        frac = count / float(1 << n)
        sample = f"integer Ryser over {count} of the 2^{n} subsets ({frac:.3g} of one permanent)"
    else:
        # direct half-range terms (O(n^2) each) over a prefix of the Gray range,
        # doubled until the sample takes about 10 s (or covers the whole range)
        T = 1 << (n - 1)
        count = min(1 << 14, T)
        while True:
            t0 = time.perf_counter()
            got = oracle.chunk_partial(A, 0, count, threads=threads)
            dt = time.perf_counter() - t0
            if dt >= 5.0 or count >= T:
                break
            grow = 2 ** max(1, min(8, int(math.log2(10.0 / max(dt, 1e-4)))))
            count = min(T, count * grow)
        frac = count / float(T)
        sample = f"{count} Gray terms formed directly (long double), {frac:.3g} of one permanent"
    value = frac * n * 2.0 ** (n - 1) / dt
    return ({"value": value, "unit": "n*2^(n-1)/s", "cores": threads, "kind": "oracle",
             "sample": sample, "seconds": round(dt, 3)}, count, got)


DTYPES = {"dd": "f64 (double-double sums)", "fp64": "f64",
          "split": "f32 products of f64 row sums, double-double sums"}
PRECISION_MODES = {"dd": 0, "fp64": 1, "split": 2}  # template argument MODE of the kernels


def oracle_check(kind, n, dA, r, count, want, precision="dd"):
    """The GPU against the oracle's sample of cpu_baseline, outside the timed
    region.  0/1: the whole permanent when the sample covers all 2^n subsets
    (Ryser's subset sum is (-1)^n per(A)), compared exactly.  Real and
    complex: perm_partial over the same Gray prefix [0, count) in the timed
    precision, the relative error of its result against the long-double sum."""
    from fractions import Fraction
    from paper_1904_06229_amd import binding as B
    if kind == "int01":
        if count != 1 << n:
            return {"range": f"{count} of the 2^{n} subsets: not a whole permanent",
                    "checked": False}
        per = want if n % 2 == 0 else -want
        return {"range": "whole permanent (all 2^%d subsets)" % n, "checked": True,
                "exact_match": per == r.exact}
    dAcm = dA.t().contiguous().t()  # the workload's matrix as a column-major view
    g = B.perm_partial(dAcm, 0, count, precision=precision)
    if kind == "complex":
        err = complex_rel_err(g, want)
    else:
        w = want.exact
        err = abs(float(Fraction(g.re_hi) + Fraction(g.re_lo) - w)) / abs(float(w))
    whole = count == 1 << (n - 1)
    return {"range": (f"whole half-range sum ({count} Gray terms)" if whole else
                      f"Gray prefix [0, {count}) of 2^{n - 1}"),
            "checked": True, "precision": precision, "rel_err_vs_oracle": err,
            "tolerance": 1e-10 if precision != "split" else None}


def gpu_qr(G):
    """Stacked reduced QR on the GPU (input generation only)."""
    import torch
    Q, R = torch.linalg.qr(torch.from_numpy(G).to("cuda"), mode="reduced")
    return Q.cpu().numpy(), R.cpu().numpy()


def exact_mean_x2(n, m):
    """E[m^n |per U_n|^2 / n!] for the n x n block of an m-mode Haar unitary:
    prod_{k<n} m/(m+k) (a soft statistical check, not from the paper)."""
    return math.prod(m / (m + k) for k in range(n))


def bench_batched(args, standalone=True, sub_frac=0.01):
    """The batched study: returns its record (and prints it when standalone).
    sub_frac: the seeded fraction of the batch checked against the oracle."""
    import numpy as np
    import torch
    from paper_1904_06229_amd import binding as B, inputs

    seed = 20190404
    t0 = time.perf_counter()
    sizes, mats = inputs.batched_haar_blocks(args.count, 8, 24, seed, qr=gpu_qr)
    gen_s = time.perf_counter() - t0
    parts, offs, o = [], [], 0
    for M in mats:
        flat = np.asfortranarray(M).ravel(order="F").view(np.float64)
        parts.append(flat)
        offs.append(o)
        o += flat.size
    dA = torch.from_numpy(np.concatenate(parts)).to("cuda")
    count = len(sizes)
    out = torch.zeros(4 * count, dtype=torch.float64, device="cuda")
    st = torch.zeros(count, dtype=torch.int32, device="cuda")
    t1 = time.perf_counter()
    if not args.no_autotune:
        B.perm_autotune(True, 8, 24)
    tune_s = time.perf_counter() - t1
    s = torch.cuda.Stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        for _ in range(args.warmup):
            B.perm_batched(dA, sizes, offs, True, out, st, stream=s, use_graph=True)
        s.synchronize()
        kms = []
        t2 = time.perf_counter()
        for _ in range(args.steps):
            ev0.record(s)
            B.perm_batched(dA, sizes, offs, True, out, st, stream=s, use_graph=True)
            ev1.record(s)
            ev1.synchronize()
            kms.append(ev0.elapsed_time(ev1))
        dt = time.perf_counter() - t2
    res = out.cpu().numpy().reshape(-1, 4)
    per = res[:, 0] + res[:, 1] + 1j * (res[:, 2] + res[:, 3])
    assert (st.cpu().numpy() == 0).all()
    steps_elem = sum(n * 2.0 ** (n - 1) for n in sizes)
    ops = sum(algorithmic_ops_per_term("complex", n) * 2.0 ** (n - 1) for n in sizes)
    kavg = sum(kms) / len(kms)
    # X^2 = m^n |per U_n|^2 / n!, m = n^2 (the paper's normalisation of S(m, n), Sec. VI)
    sz = np.array(sizes)
    x2 = np.array([(n * n) ** n * abs(p) ** 2 / math.factorial(n) for n, p in zip(sizes, per)])
    mean_check = {str(n): [float(x2[sz == n].mean()), exact_mean_x2(n, n * n)]
                  for n in (8, 16, 24)}
    edges = 10.0 ** (np.arange(-6 * 16, 2 * 16 + 1) / 16.0)  # 16 points per decade
    hist = np.histogram(np.sqrt(x2), bins=edges)[0]
    outj = {
        "metric": "batched permanents/s",
        "value": args.steps * count / dt,
        "unit": "permanents/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{count} complex Haar blocks U_n of n^2-mode unitaries, "
                               f"n uniform on 8..24, seed {seed}",
                   "element_steps_per_s": args.steps * steps_elem / dt,
                   "generate_s": round(gen_s, 2), "autotune_s": round(tune_s, 2)},
        "roofline": {"bound": "alu", "achieved": ops / (kavg * 1e-3) / 1e12,
                     "peak": PEAK_LANE_OPS / 1e12, "unit": "TOP/s",
                     "frac": ops / (kavg * 1e-3) / PEAK_LANE_OPS, "traffic": None,
                     "kernel": "batched stage+walk+finish (graph)", "kernel_ms": kavg},
        "mean_X2_vs_exact": mean_check,
        "histogram_sqrtX2_16_per_decade_nonzero": int((hist > 0).sum()),
    }
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        rng = np.random.default_rng(seed + 1)
        pick = rng.choice(count, size=max(1, int(count * sub_frac)), replace=False)
        t3 = time.perf_counter()
        worst = 0.0
        for k in pick:
            w = oracle.ryser(mats[k])
            want = complex(w.re.hi + w.re.lo, w.im.hi + w.im.lo)
            worst = max(worst, abs(per[k] - want) / abs(want))
        odt = time.perf_counter() - t3
        outj["subsample_max_rel_err"] = worst
        outj["cpu_baseline"] = {"value": len(pick) / odt, "unit": "permanents/s",
                                "cores": oracle.default_threads(), "kind": "oracle",
                                "sample": f"{len(pick)} seeded matrices ({sub_frac:.2%}) of "
                                          "the batch, long-double Ryser",
                                "seconds": round(odt, 2)}
    if standalone:
        print(json.dumps(outj))
    return outj


def bench_repeated(args):
    """n photons (48 unless --n is given) leaving an n^2-mode Haar
    interferometer two per output in n/2 outputs: per of the n x n matrix with
    n/2 distinct columns of multiplicity 2, by Eq. ryser2 (3^(n/2) terms
    instead of 2^(n-1)); with --terms-log2 K only the first 2^K terms of the
    mixed-radix Gray order (perm_repeated_partial)."""
    import numpy as np
    import torch
    from paper_1904_06229_amd import binding as B, inputs

    n, seed = args.n, 20190406
    R = n // 2
    if args.calibrate_copy:
        calibrate_copy()
    U = inputs.haar_block(n, n * n, seed)
    C = np.ascontiguousarray(U[:, :R])
    mult = [2] * R
    dC = torch.from_numpy(np.asfortranarray(C)).to("cuda")
    T = 3 ** R
    count = min(T, 2 ** args.terms_log2) if args.terms_log2 else T
    kw = {"blocks": args.blocks, "log2_chunk": args.log2_chunk}

    def call():
        if count < T:
            return B.perm_repeated_partial(dC, mult, 0, count, **kw)
        return B.perm_repeated(dC, mult, **kw)

    for _ in range(args.warmup):
        r = call()
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = call()
        kms.append(r.kernel_ms)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kavg = sum(kms) / len(kms)
    # per term: 2n row-sum updates, n-1 complex multiplies (4), weight (2), accumulate (2)
    alg = 6.0 * n * count
    desc = (f"{n}x{n} complex, {R} distinct columns x 2 (first {R} columns of the {n} x {n * n} "
            f"Haar block, seed {seed}), Eq. ryser2")
    if count < T:
        desc += f" -- PREFIX ONLY: first {count} of the {T} mixed-radix Gray terms"
    out = {
        "metric": "weighted Ryser terms/sec (n*prod(m_k+1)/s)",
        "value": args.steps * n * float(count) / dt, "unit": "n*prod(m_k+1)/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "R": R, "terms": count,
                   "inner_digits": r.log2_chunk, "blocks": r.blocks},
        "roofline": {"bound": "alu", "achieved": alg / (kavg * 1e-3) / 1e12,
                     "peak": PEAK_LANE_OPS / 1e12, "unit": "TOP/s",
                     "frac": alg / (kavg * 1e-3) / PEAK_LANE_OPS,
                     "traffic": profiled_traffic(f"mix_walk_kernel<{n}, false> (complex)", "mixed"),
                     "kernel": f"mix_walk_kernel<{n}, false> (complex)", "kernel_ms": kavg,
                     "ops_per_launch": alg},
        "result": repr(complex(r.re_hi + r.re_lo, r.im_hi + r.im_lo)),
    }
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        threads = oracle.default_threads()
        sample = 1 << 12
        while True:
            t1 = time.perf_counter()
            want = oracle.ryser2_range(C, mult, 0, sample, threads=threads)
            cdt = time.perf_counter() - t1
            if cdt >= 5.0 or sample >= T:
                break
            sample = min(T, sample * 2 ** max(1, min(8, int(math.log2(10.0 / max(cdt, 1e-4))))))
        out["cpu_baseline"] = {"value": n * sample / cdt, "unit": "n*prod(m_k+1)/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"first {sample} of the {T} Gray terms, each formed "
                                         "directly (long double)", "seconds": round(cdt, 3)}
        # the same prefix on the GPU (outside the timed region)
        g = B.perm_repeated_partial(dC, mult, 0, sample)
        out["oracle_check"] = {"range": f"mixed-radix Gray prefix [0, {sample}) of {T}",
                               "checked": True, "tolerance": 1e-10,
                               "rel_err_vs_oracle": complex_rel_err(g, want)}
    print(json.dumps(out))


def complex_rel_err(g, want):
    """|g - want| / |want| for a library result g and an oracle CPair, in exact
    rational arithmetic on the double-double parts."""
    from fractions import Fraction
    wr, wi = want.re.exact, want.im.exact
    dr = Fraction(g.re_hi) + Fraction(g.re_lo) - wr
    di = Fraction(g.im_hi) + Fraction(g.im_lo) - wi
    return math.sqrt(float(dr * dr + di * di)) / math.sqrt(float(wr * wr + wi * wi))


# LDS: 128 bytes per clock per CU (gfx950), 256 CUs, 2.4 GHz.
PEAK_LDS_BYTES = 256 * 128 * 2.4e9


def band_macs_per_row(k: int) -> int:
    """Multiply-adds of one interior row of the App. C transfer matrix as the
    kernel computes it: only masks of the surviving class (k+1 of the 2k+1
    window columns) carry terms; a mask holding column i+k takes one product,
    any other one product per column it holds."""
    top = 2 * k
    total = 0
    for m in range(1 << (2 * k + 1)):
        if bin(m).count("1") == k + 1:
            total += 1 if (m >> top) & 1 else k + 1
    return total


def bench_band(args):
    """20000 complex 64 x 64 band matrices (a_ij = 0 for |i - j| > 5), Gaussian
    entries, by the App. C transfer matrix (perm_band)."""
    import numpy as np
    import torch
    from paper_1904_06229_amd import binding as B
    from paper_1904_06229_amd import inputs

    n, k, count, seed = 64, 5, args.count if args.count != 100000 else 20000, 20190407
    if args.calibrate_copy:
        calibrate_copy()
    mats = inputs.band_batch(count, n, k, seed)
    flat = np.ascontiguousarray(np.transpose(mats, (0, 2, 1))).ravel().view(np.float64)
    dA = torch.from_numpy(flat).to("cuda")
    sizes = np.full(count, n, dtype=np.int32)
    offs = np.arange(count, dtype=np.int64) * (2 * n * n)
    out = torch.zeros(4 * count, dtype=torch.float64, device="cuda")
    st = torch.zeros(count, dtype=torch.int32, device="cuda")
    for _ in range(args.warmup):
        B.perm_band(dA, sizes, offs, k, True, out, st, blocks=args.blocks)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev0.record()
        B.perm_band(dA, sizes, offs, k, True, out, st, blocks=args.blocks)
        ev1.record()
        ev1.synchronize()
        kms.append(ev0.elapsed_time(ev1))
    dt = time.perf_counter() - t0
    assert int((st != 0).sum()) == 0
    kavg = sum(kms) / len(kms)
    macs = band_macs_per_row(k) * n * count  # interior-row count (edge rows do less)
    lds_bytes = 16.0 * macs                    # one complex coefficient read per multiply-add
    res = out.view(-1, 4)[0].cpu().numpy()
    o = {
        "metric": "band permanents/s (App. C transfer matrix)",
        "value": args.steps * count / dt, "unit": "permanents/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{count} complex 64x64 band matrices, k = 5, Ginibre entries on "
                               f"the band, seed {seed}", "n": n, "k": k, "count": count},
        "roofline": {"bound": "lds", "achieved": lds_bytes / (kavg * 1e-3) / 1e9,
                     "peak": PEAK_LDS_BYTES / 1e9, "unit": "GB/s",
                     "frac": lds_bytes / (kavg * 1e-3) / PEAK_LDS_BYTES,
                     "traffic": profiled_traffic("band_kernel<5, true>", "band"),
                     "kernel": "band_kernel<5, true>", "kernel_ms": kavg,
                     "macs_per_launch": macs},
        "result_first": repr(complex(res[0] + res[1], res[2] + res[3])),
    }
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        t1 = time.perf_counter()
        done, wants = 0, []
        while time.perf_counter() - t1 < 10.0 and done < count:
            wants.append(oracle.band(mats[done], k))
            done += 1
        cdt = time.perf_counter() - t1
        got = out.view(-1, 4)[:done].cpu().numpy()
        worst = max(complex_rel_err(SimpleNamespace(re_hi=g[0], re_lo=g[1], im_hi=g[2],
                                                    im_lo=g[3]), w)
                    for g, w in zip(got, wants))
        o["oracle_check"] = {"range": f"the first {done} matrices of the batch",
                             "checked": True, "tolerance": 1e-10,
                             "max_rel_err_vs_oracle": worst}
        o["cpu_baseline"] = {"value": done / cdt, "unit": "permanents/s", "cores": 1,
                             "kind": "oracle", "sample": f"first {done} matrices of the batch, "
                             "long-double transfer matrix, one thread", "seconds": round(cdt, 2)}
    print(json.dumps(o))


def bench_sparse(args):
    """The sparse matrices of the paper's timing study (Sec. II.D): ones on the
    diagonal, other entries 1 with probability p; n = 64, p = 0.02, exact
    0/1 result by App. B's restricted Ryser sum (64 greedy partition trials)."""
    import numpy as np
    import torch
    from paper_1904_06229_amd import binding as B

    n, p, seed, trials = 64, 0.02, 20190408, 64
    if args.calibrate_copy:
        calibrate_copy()
    r = np.random.default_rng(seed)
    M = r.random((n, n)) < p
    np.fill_diagonal(M, True)
    A = M.astype(np.uint8)
    dA = torch.from_numpy(np.asfortranarray(A)).to("cuda")
    blk, nblocks, T = B.perm_sparse_partition(dA, trials=trials, seed=1)
    for _ in range(args.warmup):
        res = B.perm_sparse(dA, trials=trials, seed=1, blocks=args.blocks)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = B.perm_sparse(dA, trials=trials, seed=1, blocks=args.blocks)
        kms.append(res.kernel_ms)
    dt = time.perf_counter() - t0
    kavg = sum(kms) / len(kms)
    alg = algorithmic_ops_per_term("real", n) * float(T)  # n updates + n-1 products + 1
    out = {
        "metric": "sparse column sets/sec (n*sets/s)",
        "value": args.steps * n * float(T) / dt, "unit": "n*sets/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64-held integers + i64 bins (exact)", "data": "synthetic",
        "config": {"workload": f"64x64 0/1, ones on the diagonal, other entries Bernoulli({p}), "
                               f"seed {seed}, exact, App. B with {trials} partition trials",
                   "n": n, "p": p, "sets": T, "blocks_in_partition": nblocks,
                   "log2_sets": math.log2(T), "inner_digits": res.log2_chunk},
        "roofline": {"bound": "alu", "achieved": alg / (kavg * 1e-3) / 1e12,
                     "peak": PEAK_LANE_OPS / 1e12, "unit": "TOP/s",
                     "frac": alg / (kavg * 1e-3) / PEAK_LANE_OPS,
                     "traffic": profiled_traffic(f"mix_exact_kernel<{n}, false>", "mixed"),
                     "kernel": f"mix_exact_kernel<{n}, false>", "kernel_ms": kavg,
                     "ops_per_launch": alg,
                     "note": "algorithmic count of the FP64 walk (2n per set); the exact "
                             "products cost more issue slots"},
        "result": str(res.exact),
    }
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        threads = oracle.default_threads()
        # the oracle's exact integer App. B sum over a prefix of its own enumeration
        # (one greedy partition trial, as perm_sparse_partial's default)
        T1 = B.perm_sparse_partition(dA)[2]  # sets of the one-trial enumeration
        count = min(1 << 12, T1)
        while True:
            t1 = time.perf_counter()
            want = oracle.sparse_range_int(A, 0, count, threads=threads)
            cdt = time.perf_counter() - t1
            if cdt >= 5.0 or count >= T1:
                break
            count = min(T1, count * 2 ** max(1, min(8, int(math.log2(10.0 / max(cdt, 1e-4))))))
        out["cpu_baseline"] = {"value": n * count / cdt, "unit": "n*sets/s", "cores": threads,
                               "kind": "oracle", "sample": f"first {count} column sets of the "
                               "Gray enumeration (one partition trial), each term formed "
                               "directly, exact integers", "seconds": round(cdt, 3)}
        g = B.perm_sparse_partial(dA, 0, count)
        out["oracle_check"] = {"range": f"Gray prefix [0, {count}) of the one-trial enumeration",
                               "checked": True, "exact_match": g.exact == want}
    print(json.dumps(out))


def bench_ensemble(args):
    """The random-ensemble study of Sec. III on the device: 100000 Ginibre
    20 x 20 matrices (resident in HBM before the timed region); a step is the
    batched permanents of all of them (perm_batched, graph replay) and the
    statistics of X = |per A| / sqrt(n!): its first four moments and F(x) on
    the 16-per-decade grid."""
    import numpy as np
    import torch
    from paper_1904_06229_amd import binding as B, ensembles, inputs

    n, seed = 20, 20190405
    count = args.count
    if args.calibrate_copy:
        calibrate_copy()
    mats = inputs.ensemble_batch("gaussian", n, count, seed)
    cm = np.ascontiguousarray(np.transpose(mats, (0, 2, 1))).astype(np.complex128)
    dA = torch.from_numpy(cm.ravel().view(np.float64)).to("cuda")
    sizes = np.full(count, n, dtype=np.int32)
    offs = np.arange(count, dtype=np.int64) * (2 * n * n)
    out = torch.zeros(4 * count, dtype=torch.float64, device="cuda")
    st = torch.zeros(count, dtype=torch.int32, device="cuda")
    t1 = time.perf_counter()
    if not args.no_autotune:
        B.perm_autotune(True, n, n)
    tune_s = time.perf_counter() - t1
    xg = ensembles.grid(1e-3, 10.0)
    norm = 1.0 / math.sqrt(math.factorial(n))
    s = torch.cuda.Stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        kms, mom, F = [], None, None
        for step in range(args.warmup + args.steps):
            if step == args.warmup:
                s.synchronize()
                t0 = time.perf_counter()
            ev0.record(s)
            B.perm_batched(dA, sizes, offs, True, out, st, stream=s, use_graph=True)
            ev1.record(s)
            o = out.view(count, 4)
            X = torch.complex(o[:, 0] + o[:, 1], o[:, 2] + o[:, 3]).abs() * norm
            mom = ensembles.moments(X)
            F = ensembles.cdf(X, xg)
            if step >= args.warmup:
                kms.append(ev0.elapsed_time(ev1))
        s.synchronize()
        dt = time.perf_counter() - t0
    assert int((st != 0).sum()) == 0
    kavg = sum(kms) / len(kms)
    ops = algorithmic_ops_per_term("complex", n) * 2.0 ** (n - 1) * count
    o = {
        "metric": "ensemble permanents/s (Sec. III study)",
        "value": args.steps * count / dt, "unit": "permanents/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{count} Ginibre {n}x{n} matrices (entries (g1 + i g2)/sqrt(2)), "
                               f"seed {seed}; per step: perm_batched + moments + F(x) on "
                               f"{len(xg)} grid points", "n": n, "count": count,
                   "autotune_s": round(tune_s, 2)},
        "roofline": {"bound": "alu", "achieved": ops / (kavg * 1e-3) / 1e12,
                     "peak": PEAK_LANE_OPS / 1e12, "unit": "TOP/s",
                     "frac": ops / (kavg * 1e-3) / PEAK_LANE_OPS,
                     "traffic": (profiled_traffic(f"batched graph, {count} x {n}x{n} complex",
                                                  "batched")),
                     "kernel": "batched stage+walk+finish (graph)", "kernel_ms": kavg},
        "moments_X": mom, "F_at_1": float(F[np.argmin(np.abs(xg - 1.0))]),
    }
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        t2 = time.perf_counter()
        done, worst = 0, 0.0
        res = out.view(count, 4).cpu().numpy()
        while time.perf_counter() - t2 < 10.0 and done < count:
            w = oracle.ryser(mats[done])
            want = complex(w.re.hi + w.re.lo, w.im.hi + w.im.lo)
            got = complex(res[done, 0] + res[done, 1], res[done, 2] + res[done, 3])
            worst = max(worst, abs(got - want) / abs(want))
            done += 1
        cdt = time.perf_counter() - t2
        o["cpu_baseline"] = {"value": done / cdt, "unit": "permanents/s",
                             "cores": oracle.default_threads(), "kind": "oracle",
                             "sample": f"first {done} matrices of the batch (long-double Ryser)",
                             "seconds": round(cdt, 2), "max_rel_err_vs_gpu": worst}
    print(json.dumps(o))


def bench_sliced(args):
    """Each step is one whole permanent as consecutive perm_partial slices
    (a progress line per slice on stderr); slice sums are added in slice order."""
    import numpy as np
    import torch
    from paper_1904_06229_amd import longrun

    kind, n, A, desc = make_workload(args.workload, args)
    dA = torch.from_numpy(np.asfortranarray(A)).to("cuda")
    slices = args.slices or 16
    kw = dict(blocks=args.blocks, log2_chunk=args.log2_chunk)
    if kind != "int01":
        kw["precision"] = args.precision

    def prog(m):
        print(m, file=sys.stderr, flush=True)

    kms, value, t_all, run_slices = [], None, 0.0, 0
    for step in range(args.warmup + args.steps):
        prog(f"step {step + 1}/{args.warmup + args.steps} ({'warmup' if step < args.warmup else 'timed'})")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        value, info = longrun.run_sliced(dA, slices=slices, progress=prog,
                                         checkpoint=args.checkpoint, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if step >= args.warmup:
            t_all += dt
            kms.extend(info["kernel_ms"])
            run_slices += len(info["kernel_ms"])
    terms = 2 ** (n - 1)
    if run_slices == 0:  # a checkpoint that was already complete: nothing was timed
        print(json.dumps({"error": "the checkpoint already holds every slice; nothing was timed",
                          "result": repr(value)}))
        sys.exit(3)
    # throughput over the slices evaluated in this run (all of them without a checkpoint)
    per_perm = n * float(terms) * run_slices / (slices * args.steps)
    alg = algorithmic_ops_per_term(kind, n) * float(terms) / slices
    kavg = sum(kms) / len(kms) if kms else float("nan")
    res = str(value.exact) if kind == "int01" else repr(value.value)
    out = {
        "metric": "Gray-code terms/sec (n*2^(n-1)/s)",
        "value": args.steps * per_perm / t_all, "unit": "n*2^(n-1)/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_all * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES.get(args.precision, "f64") if kind != "int01" else
                 "f64 exact-integer + i64 bins", "data": "synthetic",
        "config": {"workload": desc + f", whole permanent as {slices} slices of "
                                      f"{terms // slices} terms",
                   "n": n, "terms": terms, "slices": slices, "precision": args.precision,
                   "slices_timed": run_slices, "resumed": args.steps * slices - run_slices},
        "roofline": {"bound": "alu", "achieved": alg / (kavg * 1e-3) / 1e12,
                     "peak": PEAK_LANE_OPS / 1e12, "unit": "TOP/s",
                     "frac": alg / (kavg * 1e-3) / PEAK_LANE_OPS,
                     "traffic": profiled_traffic(kernel, kind),
                     "kernel": kernel, "kernel_ms": kavg,
                     "ops_per_launch": alg},
        "result": res,
    }
    if not args.no_cpu_baseline:
        cb, count, want = cpu_baseline(kind, n, A)
        out["cpu_baseline"] = cb
        out["oracle_check"] = oracle_check(kind, n, dA, None, count, want,
                                           args.precision if kind != "int01" else "dd")
    print(json.dumps(out))


def compare_precisions(fn, dA, r, timed):
    """The same whole permanent in the other precisions, once each, outside
    the timed region: their relative difference to the timed result (the
    FP64-product kernels are held to 1e-10 against each other; FP32 products
    are reported)."""
    from fractions import Fraction
    out = {}
    ref = (Fraction(r.re_hi) + Fraction(r.re_lo), Fraction(r.im_hi) + Fraction(r.im_lo))
    den = math.sqrt(float(ref[0] ** 2 + ref[1] ** 2))
    for prec in ("dd", "fp64", "split"):
        if prec == timed:
            continue
        g = fn(dA, precision=prec)
        dr = Fraction(g.re_hi) + Fraction(g.re_lo) - ref[0]
        di = Fraction(g.im_hi) + Fraction(g.im_lo) - ref[1]
        out[prec] = {"rel_diff_vs_timed": math.sqrt(float(dr * dr + di * di)) / den,
                     "kernel_ms": g.kernel_ms, "dtype": DTYPES[prec]}
    return out


def batched_leg(args):
    """The batched distribution study after the timed region: 100000 Haar
    blocks, n uniform on 8..24, autotuned, graph replay; 3 timed batches."""
    a = argparse.Namespace(**vars(args))
    a.count, a.steps, a.warmup = 100000, 3, 1
    rec = bench_batched(a, standalone=False, sub_frac=0.001)
    keep = ("value", "unit", "ms_per_step", "steps", "warmup", "config", "roofline",
            "subsample_max_rel_err", "cpu_baseline", "mean_X2_vs_exact")
    return {"metric": rec["metric"], **{k: rec[k] for k in keep if k in rec}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "c4":
        return bench_batched(args)
    if args.workload == "c6":
        return bench_repeated(args)
    if args.workload == "c7":
        return bench_band(args)
    if args.workload == "c8":
        return bench_sparse(args)
    if args.workload == "c9":
        return bench_ensemble(args)
    if args.slices or args.checkpoint or (args.workload == "c5" and not args.terms_log2):
        return bench_sliced(args)
    import numpy as np
    import torch
    from paper_1904_06229_amd import binding as B

    if args.calibrate_copy:
        calibrate_copy()
    kind, n, A, desc = make_workload(args.workload, args)
    dA = torch.from_numpy(np.ascontiguousarray(A)).to("cuda")
    fn = {"int01": B.perm_int01, "real": B.perm_real, "complex": B.perm_complex}[kind]
    # only the options that differ from the library's defaults (a plain call otherwise)
    kw = {k: v for k, v in (("blocks", args.blocks), ("log2_chunk", args.log2_chunk)) if v}
    if kind != "int01" and args.precision != "dd":
        kw["precision"] = args.precision
    terms = 2 ** (n - 1)
    if args.terms_log2:
        terms = 2 ** min(args.terms_log2, n - 1)
        desc += f" -- PREFIX ONLY: first {terms} of the 2^{n - 1} Gray terms (perm_partial)"
        dAcm = dA.t().contiguous().t()
        fn = (lambda X, **k: B.perm_partial(dAcm, 0, terms, **k))
    for _ in range(args.warmup):
        r = fn(dA, **kw)
    torch.cuda.synchronize()
    kms, calls = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = fn(dA, **kw)
        kms.append(r.kernel_ms)
        calls.append(r.total_ms)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    per_perm = n * float(terms)
    value = args.steps * per_perm / dt
    kavg = sum(kms) / len(kms)
    alg = algorithmic_ops_per_term(kind, n, getattr(r, "col0_nonzeros", 0),
                                   getattr(r, "walk_variant", 0)) * float(terms)
    achieved = alg / (kavg * 1e-3)
    kernel = f"walk_{kind}_kernel<{n}>"
    if kind != "int01" and r.walk_variant == 1:  # staging, walk and finish in one launch
        kernel = f"fused_kernel<{n}, {'true' if kind == 'complex' else 'false'}, " \
                 f"{PRECISION_MODES.get(args.precision, 0)}>"
    out = {
        "metric": "Gray-code terms/sec (n*2^(n-1)/s)",
        "value": value,
        "unit": "n*2^(n-1)/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 exact-integer + i64 bins" if kind == "int01" else
                 DTYPES.get(args.precision, "f64"),
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "terms": terms, "log2_chunk": r.log2_chunk,
                   "precision": args.precision if kind != "int01" else "exact",
                   "blocks": r.blocks, "walk_variant": r.walk_variant,
                   "col0_nonzeros": r.col0_nonzeros},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "TOP/s", "frac": achieved / PEAK_LANE_OPS,
                     "traffic": profiled_traffic(kernel, kind),
                     "kernel": kernel, "kernel_ms": kavg,
                     "ops_per_launch": alg},
    }
    # the library's own host clock per call (entry to result in host memory),
    # without the Python binding's marshalling
    out["config"]["call_ms_median"] = sorted(calls)[len(calls) // 2]
    if kind == "int01":
        out["result"] = str(r.exact)
    else:
        out["result"] = repr(r.value)
    if not args.no_cpu_baseline:
        cb, count, want = cpu_baseline(kind, n, A)
        out["cpu_baseline"] = cb
        out["oracle_check"] = oracle_check(kind, n, dA, r, count, want,
                                           args.precision if kind != "int01" else "dd")
    if kind != "int01" and not args.terms_log2 and not args.no_compare:
        out["precision_comparison"] = compare_precisions(fn, dA, r, args.precision)
    if args.workload == "c3" and not args.no_batched:
        out["batched"] = batched_leg(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
