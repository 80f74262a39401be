#!/usr/bin/env python3
"""Baryon-block benchmark on one MI355X.

A step is one pass of the whole hot path over one block of synthetic input:
the fused contraction kernel (diquark, phase-weighted third quark, MFMA
complex GEMM) plus the FP64 split-K reduction that writes B.  The default
workload is 32^3 sites, N_dil = 32 for all three quark fields, 7 momenta
(0 and the six unit vectors), complex128 inputs, one timeslice; inputs are
resident in HBM before timing starts.  All three arithmetic paths are timed;
the headline value is the FP64 path in blocks/s (the paper's arithmetic is
complex double), with the FP32 and BF16x3 split-precision paths beside it,
each with its own roofline object and its error against the oracle over the
whole block.

Usage: python bench.py [--gpus 1] [--steps K=200] [--warmup W=50] [--paths fp64,fp32,bf16x3]
                       [--workload headline-32|batched-48|uneven-32|large-64|tiny-12|projected-32|
                                   reconstruct-32|mode-triplet-32|scaling]
                       [--no-cpu-baseline] [--no-parity] [--no-graph] [--calib-copy-mib M]
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "baryon-block TFLOP/s + blocks/s, 32^3 N_dil=32: FP64 vs split-prec MFMA"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2516.6}  # dense MFMA peaks of the operand type
MFMA_PASSES = {"fp64": 1, "fp32": 1, "bf16x3": 3}
TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-5}
PREC_ID = {"fp64": 0, "fp32": 1, "bf16x3": 2}


def kernel_name(path, plan, n2, n3, zero_off=False):
    """Name of the contraction kernel a plan launches with complex128 inputs
    (as rocprofv3 lists it)."""
    z = "true" if zero_off else "false"
    if plan["kernel"] == 5:
        return "bb::f64::contract<%d, false>" % plan["nb"]
    if plan["kernel"] == 6:  # d3 blocks of 16; two row sets up to two fragments
        return "bb::f64p::contract<%d, 16, false, %s, 16, %d>" % (plan["nb"], z, 2 if plan["nb"] <= 2 else 1)
    if plan["kernel"] == 8:
        return "bb::f64p::contract<%d, 16, false, false, 4, 2>" % plan["nb"]
    if plan["kernel"] == 7:
        return "bb::f32p::contract<%d, %d, false, %s, 16>" % (plan["nb"], 32 if plan["nb"] > 2 and n3 >= 32 else 16, z)
    if plan["kernel"] == 9:
        return "bb::f32p::contract<%d, 16, false, false, 4>" % plan["nb"]
    if plan["kernel"] == 3:
        b3 = 32 if n3 >= 32 else 16
        return "bb::pord::contract<%d, %d, false, %s>" % (plan["nb"], b3, z)
    if plan["kernel"] in (2, 4):
        b2 = 32 if n2 >= 32 else 16
        return "bb::w3::contract%s<%d, %d, false>" % ("8" if plan["kernel"] == 4 else "", plan["nb"], b2)
    if plan["kernel"] == 1:
        b2, b3 = (32 if n2 >= 32 else 16), (32 if n3 >= 32 else 16)
        return "bb::fast::bb_fast<%d, %d, %d, %d, false>" % (PREC_ID[path], plan["nb"], b2, b3)
    return "bb::bb_gemm<%d, %d>" % (PREC_ID[path], plan["nb"])


def flops(V, n1, n2, n3, n_mom):
    """F_gemm: what the MFMA formulation executes (8 real flops per complex
    multiply-add over K = 3V, M = n1 n2, N = n3 n_mom).  F_alg: the paper's
    operation order (diquark, singlet, momentum projection)."""
    f_gemm = 24.0 * n_mom * V * n1 * n2 * n3
    f_alg = 42.0 * V * n1 * n2 + (22.0 + 8.0 * n_mom) * V * n1 * n2 * n3
    return f_gemm, f_alg


# Sources each contraction kernel family is compiled from (a change to any
# of them invalidates counter figures taken before it).
KERNEL_SOURCES = {
    "bb::w3::": ("bb_w3.hip", "bb_fast.h", "bb_internal.h"),
    "bb::fast::": ("bb_fast.h", "bb_fast_fp32.hip", "bb_fast_bf16.hip", "bb_internal.h"),
    "bb::pord::": ("bb_pord.hip", "bb_fast.h", "bb_internal.h"),
    "bb::bb_gemm": ("bb_kernels.hip", "bb_internal.h"),
    "bb::bb_reduce": ("bb_kernels.hip", "bb_internal.h"),
    "bb::f64::": ("bb_f64.hip", "bb_internal.h"),
    "bb::f64p::": ("bb_f64p.hip", "bb_fast.h", "bb_internal.h"),
    "bb::f32p::": ("bb_f32p.hip", "bb_fast.h", "bb_internal.h"),
}


def sources_of(kname: str):
    for prefix, files in KERNEL_SOURCES.items():
        if kname.startswith(prefix):
            return files
    raise KeyError(kname)


def executed_flops(path, plan, V, n, n_mom, zero_off=False):
    """FP flops one headline launch executes on the pipes its roofline prices.
    Fused kernels: the complex GEMM on the matrix cores (F_gemm = 24 n_mom V
    n^3, 8 real flops per complex multiply-add), three times over for the
    three BF16 products of BF16x3; FP64 kernel 5 forms each complex product
    from three real products (6 real flops per complex multiply-add): 3/4 of
    F_gemm.  Paper-order kernels: the momentum projection on the matrix
    cores (6 flops per padded momentum with three real products: FP64
    kernels 6 and 8, FP32 kernels 7 and 9 up to two fragments; 8 with four
    for FP32 above), plus for the FP64
    kernels their vector work, the diquark (42 V n^2) and the singlet with
    its Re + Im (23 V n^3): FP64 vector and matrix work share one 78.6
    TFLOP/s issue rate on gfx950 and never overlap, so both count against
    that peak.  zero_off: kernels 6 and 7 project n_mom - 1 momenta (the
    zero one is summed on the vector unit)."""
    k, nb = plan["kernel"], plan["nb"]
    vn3 = float(V) * n ** 3
    m = n_mom - (1 if zero_off else 0)
    if k == 5:
        return 0.75 * 24.0 * n_mom * vn3
    if k in (6, 8):
        w = 16 if k == 6 else 4
        padded = -(-m // (w * nb)) * w * nb
        return 6.0 * padded * vn3 + 23.0 * vn3 + 42.0 * V * n * n
    if k in (7, 9):  # three real products up to two fragments, four above
        w = 16 if k == 7 else 4
        padded = -(-m // (w * nb)) * w * nb
        return (6.0 if nb <= 2 else 8.0) * padded * vn3
    return MFMA_PASSES[path] * 24.0 * n_mom * vn3


def flops_note(path, plan):
    k = plan["kernel"]
    if k == 5:
        return "18 n_mom V n^3: three real products per complex multiply-add on the matrix cores"
    if k in (6, 8):
        return ("6 n_pad V n^3 on the matrix cores (the momentum projection with three real products, n_pad the "
                "momenta padded to fragments of %d) + 23 V n^3 + 42 V n^2 on the vector unit (singlet, diquark), "
                "one FP64 issue rate" % (16 if k == 6 else 4))
    if k in (7, 9):
        pad = "n_pad the momenta padded to fragments of %d" % (16 if k == 7 else 4)
        return ("6 n_pad V n^3: the momentum projection with three real products, " + pad if plan["nb"] <= 2 else
                "8 n_pad V n^3: the momentum projection with four real products, " + pad)
    return "%d x 24 n_mom V n^3" % MFMA_PASSES[path]


class no_gc:
    """Python's cyclic garbage collector paused over a timed region: a full
    collection in a process holding torch takes milliseconds, long enough to
    drain the GPU queue between two launches."""

    def __enter__(self):
        gc.collect()
        self.was = gc.isenabled()
        gc.disable()

    def __exit__(self, *exc):
        if self.was:
            gc.enable()


def kernel_source_sha(files) -> str:
    """Hash of the code a kernel is compiled from (comments and layout
    removed): counter figures taken for another hash no longer describe the
    kernel that runs."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2211_16278_amd", "csrc")
    for f in files:
        with open(os.path.join(csrc, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def read_traffic(path_name: str, workload: str, kname: str):
    """HBM bytes of a path from the committed counter summary: (bytes per
    launch of the contraction kernel, bytes of the whole step, the minimal
    bytes of one block).  A figure is None when there is no summary, it is
    of another kernel, or a kernel's sources changed since the counters were
    taken."""
    fn = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (path_name, workload))
    if not os.path.exists(fn):
        return None, None, None
    with open(fn) as f:
        rec = json.load(f)
    if rec.get("kernel") != kname or rec.get("kernel_source_sha") != kernel_source_sha(sources_of(kname)):
        return None, None, rec.get("minimal_block_bytes")
    step = rec.get("step_kernels")
    step_bytes = None
    if step and all(k["kernel_source_sha"] == kernel_source_sha(sources_of(k["kernel"])) for k in step):
        step_bytes = sum(k["hbm_bytes_per_step"] for k in step)
    return rec.get("hbm_bytes_per_launch"), step_bytes, rec.get("minimal_block_bytes")


def device_fields(torch, dev, shape_list, dtype, seed):
    """Seeded iid complex-normal fields generated on the device (the batched
    workloads hold tens of GB of inputs; content does not affect timing)."""
    g = torch.Generator(device=dev)
    g.manual_seed(16278 * 1000 + seed)
    real = torch.float32 if dtype == "c64" else torch.float64
    out = []
    for shp in shape_list:
        t = torch.empty((*shp, 2), dtype=real, device=dev)
        t.normal_(0.0, 0.5 ** 0.5, generator=g)
        out.append(torch.view_as_complex(t))
    return out


def zero_on_vector_unit(plan, mom, L):
    """Kernels 6 and 7 sum the zero momentum (mod L) of a set of 16 k + 1 > 1
    momenta on the vector unit and project only the other 16 k on the
    matrix cores; kernel 3 with one fragment does so at 32 k + 1."""
    n = len(mom)
    skips = (plan["kernel"] in (6, 7) and n % 16 == 1) or (plan["kernel"] == 3 and plan["nb"] == 1 and n % 32 == 1)
    return n > 1 and skips and any(all(int(c) % L == 0 for c in m) for m in mom)


def mfma_flops(plan, V, n1, n2, n3, n_mom, zero_off=False):
    """Flops of one MFMA pass of the formulation a plan runs: the fused GEMM
    (24 n_mom V n1 n2 n3; 18 for FP64 kernel 5's three real products) or, for
    the paper-order kernels, only the momentum projection (8 n_mom V n1 n2 n3
    for kernels 3, 7 and 9 (6 for 7 and 9 up to two fragments), 6 for FP64
    kernels 6 and 8; their singlet runs on the
    vector unit), over n_mom - 1 momenta when the zero one is summed on the
    vector unit (zero_off)."""
    per = {3: 8.0, 5: 18.0, 6: 6.0, 7: 6.0 if plan["nb"] <= 2 else 8.0, 8: 6.0,
           9: 6.0 if plan["nb"] <= 2 else 8.0}.get(plan["kernel"], 24.0)
    return per * (n_mom - (1 if zero_off else 0)) * V * n1 * n2 * n3


def batch_workload(torch, dev, name):
    """Descriptors (q1, q2, q3, out) of a grouped workload, all resident on the device."""
    from paper_2211_16278_amd import synth
    wl = synth.WORKLOADS[name]
    L, T = wl["L"], wl["T"]
    V = L ** 3
    mom = synth.momenta(wl["momenta"])
    descs, fields, f_gemm, f_alg = [], [], 0.0, 0.0
    if name == "batched-48":
        # 3 quark lines x 4 spin components per timeslice; spin triples (s, s, s).
        n = wl["ndil"]
        for t in range(T):
            lines = [device_fields(torch, dev, [(V, 3, n)] * 4, wl["dtype"], 100 * t + ln) for ln in range(3)]
            fields.append(lines)
            for s_ in range(4):
                out = torch.empty((len(mom), n, n, n), dtype=torch.complex128, device=dev)
                descs.append((lines[0][s_], lines[1][s_], lines[2][s_], out))
    elif name == "uneven-32":
        # 8 noise triples per timeslice with N_dil (16, 32, 64)[k mod 3], 3 lines x 4
        # spins each; the first 20 spin triples of {0..3}^3 per noise triple.
        import itertools
        triples = list(itertools.product(range(4), repeat=3))[:20]
        for t in range(T):
            for k in range(8):
                n = (16, 32, 64)[k % 3]
                lines = [device_fields(torch, dev, [(V, 3, n)] * 4, wl["dtype"], 10000 * t + 100 * k + ln)
                         for ln in range(3)]
                fields.append(lines)
                for (a, b, c) in triples:
                    out = torch.empty((len(mom), n, n, n), dtype=torch.complex128, device=dev)
                    descs.append((lines[0][a], lines[1][b], lines[2][c], out))
    elif name == "projected-32":
        # 3 quark lines x 4 spin components per timeslice; the spin-triple
        # terms of synth.PROJECTION_TERMS summed into 2 outputs per timeslice.
        n = wl["ndil"]
        for t in range(T):
            lines = [device_fields(torch, dev, [(V, 3, n)] * 4, wl["dtype"], 100 * t + ln) for ln in range(3)]
            fields.append(lines)
            outs = [torch.empty((len(mom), n, n, n), dtype=torch.complex128, device=dev) for _ in range(2)]
            for g, (a, b, c), coef in synth.PROJECTION_TERMS:
                descs.append((lines[0][a], lines[1][b], lines[2][c], outs[g]))
    elif name in ("large-64", "tiny-12", "headline-32"):
        n = wl["ndil"]
        for t in range(T):
            q = device_fields(torch, dev, [(V, 3, n)] * 3, wl["dtype"], t)
            fields.append(q)
            out = torch.empty((len(mom), n, n, n), dtype=torch.complex128, device=dev)
            descs.append((q[0], q[1], q[2], out))
    else:
        raise SystemExit("unknown workload %s" % name)
    for q1, q2, q3, _ in descs:
        fg, fa = flops(V, q1.shape[-1], q2.shape[-1], q3.shape[-1], len(mom))
        f_gemm += fg
        f_alg += fa
    return L, mom, descs, fields, f_gemm, f_alg, wl


def workspace_gib(args, name):
    if args.workspace_gib is not None:
        return args.workspace_gib
    return {"uneven-32": 128, "batched-48": 40, "large-64": 40}.get(name, 16)


def run_batch_workload(args, name):
    """Time a grouped workload: a step is one grouped launch over all its blocks."""
    import torch
    from paper_2211_16278_amd import binding, synth
    dev = torch.device("cuda:0")
    L, mom, descs, fields, f_gemm, f_alg, wl = batch_workload(torch, dev, name)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    max_n = max(max(d[0].shape[-1], d[1].shape[-1], d[2].shape[-1]) for d in descs)
    res = {}
    for pname in [p for p in args.paths.split(",") if p]:
        bb = binding.BaryonBlocks(L, prec=pname, in_dtype=wl["dtype"], max_ndil=max_n, stream=stream,
                                  workspace_cap=workspace_gib(args, name) << 30)
        # The step's launches (W images, contraction, reduction) are captured
        # once into a hipGraph and replayed.
        bb.set_graph(not args.no_graph)
        if name == "projected-32":
            coefs = [c for _, _, c in synth.PROJECTION_TERMS] * wl["T"]
            step = lambda: bb.compute_projected(descs, coefs, mom)  # noqa: E731
        else:
            step = lambda: bb.compute_batch(descs, mom)  # noqa: E731
        with no_gc():  # collected once, before the warmup (no idle pause before the timed steps)
            for _ in range(args.warmup):
                step()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record(stream)
            for _ in range(args.steps):
                step()
            e1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        step_ms = max(e0.elapsed_time(e1), wall * 1e3) / args.steps
        bb.profile(True)
        bb.profile_read()
        step()
        gemm_ms, red_ms, prep_ms, launches = bb.profile_read()
        bb.profile(False)
        f_mfma, kernels = 0.0, set()
        for q1, q2, q3, _ in descs:
            shp = (q1.shape[-1], q2.shape[-1], q3.shape[-1], len(mom))
            plan = bb.get_plan(*shp)
            kernels.add(plan["kernel"])
            f_mfma += mfma_flops(plan, L ** 3, *shp, zero_off=zero_on_vector_unit(plan, mom, L))
        bb.close()
        err = None
        if name != "projected-32" and not args.no_parity:
            # Sampled parity: 64 seeded entries (every momentum) of the first,
            # the middle and the last block against the oracle.
            import numpy as np
            import oracle
            g = np.random.default_rng(11)
            err = 0.0
            for i in sorted({0, len(descs) // 2, len(descs) - 1}):
                q1, q2, q3, o = descs[i]
                ns = (q1.shape[-1], q2.shape[-1], q3.shape[-1])
                ents = np.stack([g.integers(0, k, 64) for k in ns], axis=1).astype(np.int32)
                host = [q.cpu().numpy().astype(np.complex128) for q in (q1, q2, q3)]
                ref = oracle.bblock_entries(L, *host, mom, ents)
                idx = torch.from_numpy(ents.astype(np.int64)).to(dev)
                got = o[:, idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
                err = max(err, float(np.abs(got - ref).max() / np.abs(ref).max()))
                del host
        if name == "projected-32" and not args.no_parity:
            # Sampled parity of output 0 of timeslice 0 against the oracle's sum of blocks.
            import numpy as np
            import oracle
            rows = np.array([[0, 0], [31, 31], [7, 19]], dtype=np.int32)
            terms = [(i, tr) for i, (g, tr, _) in enumerate(synth.PROJECTION_TERMS) if g == 0]
            host = [[f.cpu().numpy() for f in line] for line in fields[0]]
            trip = [(host[0][a], host[1][b], host[2][c]) for _, (a, b, c) in terms]
            ref = oracle.bblock_rows_projected(L, trip, [coefs[i] for i, _ in terms], mom, rows)
            got = descs[terms[0][0]][3].cpu().numpy()
            sub = np.stack([got[:, d1, d2, :] for d1, d2 in rows], axis=1)
            err = float(np.abs(sub - ref).max() / np.abs(ref).max())
        res[pname] = {"blocks_per_s": len(descs) * 1e3 / step_ms, "ms_per_step": step_ms,
                      "tflops_gemm_count": f_gemm / (step_ms * 1e-3) / 1e12,
                      "tflops_paper_count": f_alg / (step_ms * 1e-3) / 1e12,
                      "contraction_kernel_ms_per_step": gemm_ms, "reduce_kernel_ms_per_step": red_ms,
                      "w_image_kernel_ms_per_step": prep_ms,
                      "contraction_launches_per_step": launches,
                      "graph_replayed": not args.no_graph,
                      "kernels": sorted(kernels),
                      "mfma_frac": MFMA_PASSES[pname] * f_mfma / (gemm_ms * 1e-3) / 1e12 / PEAK_TFLOPS[pname],
                      "gemm_equivalent_frac": MFMA_PASSES[pname] * f_gemm / (gemm_ms * 1e-3) / 1e12
                      / PEAK_TFLOPS[pname],
                      "err_max_sampled": err}
        print("# %s %-6s %d blocks  %.2f ms/step  %.1f blocks/s  kernels %s  MFMA %.1f%% (fused-GEMM equivalent "
              "%.1f%%)  reduce/combine %.2f ms%s" % (
            name, pname, len(descs), step_ms, len(descs) * 1e3 / step_ms, sorted(kernels),
            100 * res[pname]["mfma_frac"], 100 * res[pname]["gemm_equivalent_frac"], red_ms,
            "  err %.2e" % err if err is not None else ""), file=sys.stderr, flush=True)
    head = "bf16x3" if "bf16x3" in res else next(iter(res))
    rec = {"metric": METRIC, "value": res[head]["blocks_per_s"], "unit": "blocks/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": res[head]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": head,
           "data": "synthetic (seeded iid complex normal quark fields, generated on the device)",
           "config": {"workload": name, "L": L, "T": wl["T"], "n_dil": wl["ndil"], "n_mom": len(mom),
                      "blocks_per_step": len(descs), "in_dtype": wl["dtype"]},
           "paths": res}
    print(json.dumps(rec), flush=True)
    return 0


def run_mode_workload(args, name):
    """LapH-subspace workloads (Sec. 2 of the paper).

    reconstruct-32: eq. (2) for 12 coefficient sets (3 quark lines x 4 spin
      components) of N_dil = 32 rows on 128 eigenvectors of a 32^3 timeslice,
      one FP64 complex GEMM (M = 3V, N = 384, K = 128); a step is one call,
      the value is reconstructed fields (coefficient sets) per second.
    mode-triplet-32: the mode triplets of eq. (4) for 64 eigenvectors and
      7 momenta are built once (BF16X3 block kernels, timed as setup); a step
      is one batched contraction of 16 coefficient triples (N_dil = 32) onto
      them (three FP64 complex GEMMs), the value is blocks per second; one
      triple per call is timed beside it."""
    import numpy as np
    import torch
    from paper_2211_16278_amd import binding, synth
    from oracle import modes
    dev = torch.device("cuda:0")
    wl = synth.WORKLOADS[name]
    L, n_ev, n_dil = wl["L"], wl["n_ev"], wl["ndil"]
    V = L ** 3
    stream = torch.cuda.current_stream()
    bb = binding.BaryonBlocks(L, prec="bf16x3", in_dtype=wl["dtype"], max_ndil=n_ev, stream=stream,
                              workspace_cap=workspace_gib(args, name) << 30)
    phi_h = synth.laplacian_modes(L, n_ev, workload=50)
    phi = torch.from_numpy(phi_h).to(dev)
    extra, err = {}, None
    if name == "reconstruct-32":
        n_q = wl["n_q"]
        Q_h = synth.coefficients(n_q, n_dil, n_ev, workload=50)
        Q = torch.from_numpy(Q_h).to(dev)
        dt = torch.complex64 if wl["dtype"] == "c64" else torch.complex128
        q = torch.empty((n_q, V, 3, n_dil), dtype=dt, device=dev)
        step = lambda: bb.reconstruct(phi, Q, out=q)  # noqa: E731
        flops = 8.0 * 3 * V * n_ev * n_dil * n_q
        nbytes = 3 * V * n_ev * 16 + n_q * n_dil * n_ev * 16 + q.numel() * q.element_size()
        units, unit = n_q, "fields/s"
        kernel = "bb::zg::zgemm<2, 2>"
    else:
        mom = synth.momenta(wl["momenta"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T = bb.mode_triplets(phi.to(torch.complex64) if wl["dtype"] == "c64" else phi, mom)
        torch.cuda.synchronize()
        extra["setup_ms"] = (time.perf_counter() - t0) * 1e3
        n_c = wl["n_c"]
        Qs_h = [synth.coefficients(n_c, n_dil, n_ev, workload=51, role=i) for i in range(3)]
        Qs = [torch.from_numpy(x).to(dev) for x in Qs_h]
        B = torch.empty((n_c, len(mom), n_dil, n_dil, n_dil), dtype=torch.complex128, device=dev)
        step = lambda: bb.mode_contract_batch(T, *Qs, out=B)  # noqa: E731
        n_mom = len(mom)
        flops = 8.0 * n_c * n_mom * (n_dil * n_ev ** 3 + n_dil ** 2 * n_ev ** 2 + n_dil ** 3 * n_ev)
        nbytes = T.numel() * 16 + 3 * n_c * n_dil * n_ev * 16 + B.numel() * 16
        units, unit = n_c, "blocks/s"
        kernel = "bb::zg::zgemm (3 launches: l1, l2, l3)"
        # One triple per call, for comparison.
        B1 = torch.empty((len(mom), n_dil, n_dil, n_dil), dtype=torch.complex128, device=dev)
        single = lambda: bb.mode_contract(T, *[q[0] for q in Qs], out=B1)  # noqa: E731
        with no_gc():
            for _ in range(args.warmup):
                single()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                single()
            torch.cuda.synchronize()
            extra["single_triple_blocks_per_s"] = args.steps / (time.perf_counter() - t0)
    with no_gc():  # collected once, before the warmup (no idle pause before the timed steps)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    step_ms = max(e0.elapsed_time(e1), wall * 1e3) / args.steps
    bb.profile(True)
    bb.profile_read()
    n_prof = min(args.steps, 50)
    for _ in range(n_prof):
        step()
    gemm_ms, _, _, launches = bb.profile_read()
    bb.profile(False)
    k_ms = gemm_ms / n_prof
    if not args.no_parity:
        if name == "reconstruct-32":
            xs = np.array([0, 1, V // 3, V - 1])
            ref = modes.reconstruct(Q_h, phi_h[xs])
            got = q[:, torch.from_numpy(xs).to(dev)].cpu().numpy()
        else:
            ref = modes.mode_contract(*[q[n_c - 1] for q in Qs_h], T.cpu().numpy())
            got = B[n_c - 1].cpu().numpy()
        err = float(np.abs(got - ref).max() / np.abs(ref).max())
    bb.close()
    ach = flops / (k_ms * 1e-3) / 1e12
    print("# %s  %.3f ms/step  %.1f %s  kernels %.3f ms (%d launches)  FP64 MFMA %.1f TF (%.1f%%)%s%s" % (
        name, step_ms, units * 1e3 / step_ms, unit, k_ms, launches // n_prof, ach, 100 * ach / PEAK_TFLOPS["fp64"],
        "  setup %.1f ms" % extra["setup_ms"] if "setup_ms" in extra else "",
        "  err %.2e" % err if err is not None else "") + (
        "  (one triple per call: %.1f blocks/s)" % extra["single_triple_blocks_per_s"]
        if "single_triple_blocks_per_s" in extra else ""), file=sys.stderr, flush=True)
    rec = {"metric": unit.replace("/s", "") + " per second, " + name, "value": units * 1e3 / step_ms, "unit": unit,
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded iid complex normal eigenvector stand-ins and coefficients)",
           "config": {"workload": name, "L": L, "n_ev": n_ev, "n_dil": n_dil,
                      **({"n_q": wl["n_q"], "out_dtype": wl["dtype"]} if name == "reconstruct-32"
                         else {"n_mom": len(mom), "triples_per_call": wl["n_c"], "triplet_prec": "bf16x3"})},
           "roofline": {"bound": "mfma", "kernel": kernel, "achieved": ach, "peak": PEAK_TFLOPS["fp64"],
                        "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS["fp64"], "traffic": None,
                        "flops_per_step": flops, "algorithmic_bytes_per_step": nbytes,
                        "hbm_GBps_at_kernel_time": nbytes / (k_ms * 1e-3) / 1e9},
           "kernel_ms_per_step": k_ms, "err_max_sampled": err, **extra}
    print(json.dumps(rec), flush=True)
    return 0


def run_scaling(args):
    """Problem-size scaling (the GPU analogue of the paper's Sec. 4 scan over
    volume and dilution size): time per block of one timeslice, 7 momenta,
    complex128 inputs, against N_dil (L = 32) and against L (N_dil = 32).  The
    cost of eq. (3) is O(V N_dil^3), so time / (V N_dil^3) should be flat once
    the device is saturated; the value is the largest deviation from the
    reference point (L = 32, N_dil = 32) over the saturated points."""
    import torch
    from paper_2211_16278_amd import binding, synth
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    mom = synth.momenta("axis")
    points = [(32, n) for n in (16, 24, 32, 40, 48, 64)] + [(L, 32) for L in (16, 24, 40, 48)]
    res = {}
    for pname in [p for p in args.paths.split(",") if p]:
        rows = []
        for L, n in points:
            qs = device_fields(torch, dev, [(L ** 3, 3, n)] * 3, "c128", 7 * L + n)
            out = torch.empty((1, len(mom), n, n, n), dtype=torch.complex128, device=dev)
            with binding.BaryonBlocks(L, prec=pname, in_dtype="c128", max_ndil=64, stream=stream) as bb:
                step = lambda: bb.compute(*qs, mom, out=out)  # noqa: E731
                for _ in range(max(2, args.warmup // 10)):
                    step()
                torch.cuda.synchronize()
                k = max(5, args.steps // 10)
                with no_gc():
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(k):
                        step()
                    e1.record(stream)
                    torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / k
            rows.append({"L": L, "n_dil": n, "ms_per_block": ms, "ns_per_unit": ms * 1e6 / (L ** 3 * n ** 3)})
            del qs, out
        ref = next(r["ns_per_unit"] for r in rows if r["L"] == 32 and r["n_dil"] == 32)
        for r in rows:
            r["relative"] = r["ns_per_unit"] / ref
        sat = [r for r in rows if r["L"] >= 24 and r["n_dil"] >= 24]
        dev_max = max(abs(r["relative"] - 1.0) for r in sat)
        res[pname] = {"points": rows, "max_deviation_saturated": dev_max}
        print("# scaling %-6s " % pname + "  ".join("L%d/N%d %.3f" % (r["L"], r["n_dil"], r["relative"]) for r in rows)
              + "  max dev (L, N_dil >= 24) %.3f" % dev_max, file=sys.stderr, flush=True)
    head = "bf16x3" if "bf16x3" in res else next(iter(res))
    rec = {"metric": "max deviation of time/(V N_dil^3) from the 32^3, N_dil=32 point (saturated sizes)",
           "value": res[head]["max_deviation_saturated"], "unit": "fraction", "n_gpus": 1,
           "steps": max(5, args.steps // 10), "warmup": max(2, args.warmup // 10), "ms_per_step": None,
           "higher_is_better": False, "scaling": "problem size", "vs_baseline": None, "dtype": head,
           "data": "synthetic (seeded iid complex normal quark fields, generated on the device)",
           "config": {"workload": "scaling: L=32 with N_dil 16..64, N_dil=32 with L 16..48, 7 momenta, c128"},
           "paths": res}
    print(json.dumps(rec), flush=True)
    return 0


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2]


def _rows_rate(oracle, L, qs, mom, rows, reps=3):
    """Median over reps of seconds per (d1, d2) row of the oracle's rows variant."""
    import numpy as np
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        oracle.bblock_rows(L, *qs, mom, np.asarray(rows, dtype=np.int32))
        times.append((time.perf_counter() - t0) / len(rows))
    return _median(times)


def cpu_baseline(L, qs, mom, M):
    """The oracle, untuned, on the host cores: the whole headline block on all
    threads and a row sample on one thread (median of 3 each), and the
    per-block oracle time of the other workloads' block shapes extrapolated
    from row samples on all threads (time per row x rows per block)."""
    import numpy as np
    import oracle
    from paper_2211_16278_amd import synth
    all_threads = oracle.max_threads()
    n2 = qs[1].shape[2]
    t_start = time.perf_counter()
    # All threads, whole block, median of 3.
    full = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.bblock(L, *qs, mom)
        full.append(time.perf_counter() - t0)
    t_all = _median(full)
    # One thread: 48 rows (of 1024), median of 3, scaled to the block.
    oracle.set_threads(1)
    try:
        rows1 = [[r // n2, r % n2] for r in range(0, M, max(1, M // 48))][:48]
        t_row1 = _rows_rate(oracle, L, qs, mom, rows1)
    finally:
        oracle.set_threads(all_threads)
    t_one = t_row1 * M
    # Other block shapes, all threads: one row per thread, one run each.
    extrap = {}
    shapes = [("batched-48", 48, 32, "cube", 192), ("uneven-32 N_dil 16", 32, 16, "axis", 960),
              ("uneven-32 N_dil 32", 32, 32, "axis", 960), ("uneven-32 N_dil 64", 32, 64, "axis", 640),
              ("large-64", 64, 64, "shell4", 4)]
    for name, Lx, n, mset, blocks in shapes:
        qx = synth.gaussian_fields(Lx, (n, n, n), workload=90)
        mx = synth.momenta(mset)
        rows = [[(7 * i) % n, (3 * i + 1) % n] for i in range(all_threads)]
        per_row = _rows_rate(oracle, Lx, qx, mx, rows, reps=1)
        extrap[name] = {"L": Lx, "n_dil": n, "n_mom": len(mx), "s_per_block": per_row * n * n,
                        "blocks_in_workload": blocks, "s_workload": per_row * n * n * blocks}
        del qx
    return {"value": 1.0 / t_all, "unit": "blocks/s", "cores": all_threads, "kind": "oracle",
            "sample": "whole 32^3 N_dil 32 block (7 momenta) on %d threads, median of 3 runs (%.2f s each); "
                      "1 thread: %d of %d (d1,d2) rows, median of 3, scaled to the block" % (
                          all_threads, t_all, len(rows1), M),
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "all_threads": {"threads": all_threads, "s_per_block": t_all, "blocks_per_s": 1.0 / t_all,
                            "runs_s": full},
            "one_thread": {"threads": 1, "s_per_block": t_one, "blocks_per_s": 1.0 / t_one,
                           "rows_timed": len(rows1)},
            "extrapolated_other_workloads": {"note": "EXTRAPOLATED: time per (d1,d2) row on all threads "
                                                     "(one run over %d rows) x rows per block x blocks"
                                                     % all_threads, **extrap},
            "wall_s": time.perf_counter() - t_start}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--paths", default="fp64,fp32,bf16x3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="always launch eagerly (default: the library's choice, hipGraph replay for schedules of 4 "
                         "or more launches)")
    ap.add_argument("--workload", default="headline-32",
                    help="headline-32 (the benchmark line), or a grouped workload: batched-48, uneven-32, "
                         "large-64, tiny-12, projected-32 (spin projection), or a LapH-subspace workload: "
                         "reconstruct-32 (eq. (2)), mode-triplet-32 (eq. (4) route), or scaling (time per "
                         "block against volume and dilution size)")
    ap.add_argument("--workspace-gib", type=int, default=None,
                    help="library workspace cap (default: 128 for uneven-32, whose W images of one step's 512 distinct "
                         "third fields, 105 GB, then stay resident; 40 for batched-48 and large-64, whose split partials "
                         "(34 and 16.5 GiB in BF16X3 and FP32) then fit one launch; 16 otherwise)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, run one plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (blocks shard across GPUs with no "
              "communication). Run with --gpus 1.", file=sys.stderr)
        return 2

    if args.workload == "scaling":
        return run_scaling(args)
    if args.workload in ("reconstruct-32", "mode-triplet-32"):
        return run_mode_workload(args, args.workload)
    if args.workload != "headline-32":
        return run_batch_workload(args, args.workload)

    import numpy as np
    import torch

    from paper_2211_16278_amd import binding, synth

    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    wl = synth.WORKLOADS["headline-32"]
    L, n = wl["L"], wl["ndil"]
    V = L ** 3
    mom = synth.momenta(wl["momenta"])
    n_mom = len(mom)
    qs = synth.gaussian_fields(L, (n, n, n), workload=2)
    tq = [torch.from_numpy(q).to(dev) for q in qs]
    out = torch.empty((1, n_mom, n, n, n), dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    f_gemm, f_alg = flops(V, n, n, n, n_mom)
    stream = torch.cuda.current_stream()

    ref_block = None
    if not args.no_parity:
        import oracle
        ref_block = oracle.bblock(L, *qs, mom)  # every entry is compared

    paths = {}
    for pname in [p for p in args.paths.split(",") if p]:
        bb = binding.BaryonBlocks(L, prec=pname, in_dtype="c128", max_ndil=n, stream=stream)
        if args.no_graph:
            bb.set_graph(False)
        plan = bb.get_plan(n, n, n, n_mom)
        # The collector runs once, before the warmup: a collection between
        # the warmup and the timed steps leaves the GPU idle for tens of ms,
        # and the first steps after such a pause run at lower clocks.
        with no_gc():
            for _ in range(args.warmup):
                bb.compute(*tq, mom, out=out)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record(stream)
            for _ in range(args.steps):
                bb.compute(*tq, mom, out=out)
            e1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            # Per-step durations: an event pair around every step of a second pass.
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(args.steps)]
            for a, b in evs:
                a.record(stream)
                bb.compute(*tq, mom, out=out)
                b.record(stream)
            torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        per_step = sorted(a.elapsed_time(b) for a, b in evs)
        # Per-kernel durations: HIP events around each launch on the library's stream.
        bb.profile(True)
        bb.profile_read()
        for _ in range(args.steps):
            bb.compute(*tq, mom, out=out)
        gemm_ms, red_ms, prep_ms, launches = bb.profile_read()
        bb.profile(False)
        err = None
        if ref_block is not None:
            err = float(np.abs(out[0].cpu().numpy() - ref_block).max() / np.abs(ref_block).max())
        bb.close()
        step_ms = max(ms, wall * 1e3) / args.steps
        g_avg = gemm_ms / max(1, launches)
        f_exec = executed_flops(pname, plan, L ** 3, n, len(mom), zero_on_vector_unit(plan, mom, L))
        # The FP64 paper-order kernels price the paper's own operation count
        # (F_alg: diquark, singlet, projection, 8 flops per complex
        # multiply-add, no padding) against the FP64 issue rate their matrix
        # and vector work share; the others their executed MFMA flops.
        paper_order = plan["kernel"] in (6, 8)
        f_roof = f_alg if paper_order else f_exec
        ach = f_roof / (g_avg * 1e-3) / 1e12
        kname = kernel_name(pname, plan, n, n, zero_on_vector_unit(plan, mom, L))
        # HBM bytes from the committed counters; the minimal bytes of a block
        # are its inputs read once and its output written once.
        traffic, step_traffic, minimal_bytes = read_traffic(pname, "headline-32", kname)
        paths[pname] = {
            "blocks_per_s": 1e3 / step_ms,
            "ms_per_step": step_ms,
            "event_ms_per_step": ms / args.steps,
            "wall_ms_per_step": wall * 1e3 / args.steps,
            "step_ms_min_median_max": [per_step[0], per_step[len(per_step) // 2], per_step[-1]],
            "tflops_gemm_count": f_gemm / (step_ms * 1e-3) / 1e12,
            "tflops_paper_count": f_alg / (step_ms * 1e-3) / 1e12,
            "contraction_kernel_ms": g_avg,
            "reduce_kernel_ms": red_ms / max(1, launches),
            "w_image_kernel_ms": prep_ms / max(1, launches),
            "outside_kernels_ms": per_step[len(per_step) // 2] - (gemm_ms + red_ms + prep_ms) / max(1, launches),
            "err_max": err,
            "err_entries_compared": None if err is None else int(ref_block.size),
            "tol": TOL[pname],
            "plan": plan,
            "roofline": {"bound": "mfma", "kernel": kname, "achieved": ach, "peak": PEAK_TFLOPS[pname],
                         "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS[pname],
                         "step_frac": f_roof / (step_ms * 1e-3) / 1e12 / PEAK_TFLOPS[pname],
                         "traffic": traffic,
                         "step_traffic": step_traffic,
                         "minimal_bytes": minimal_bytes,
                         "flops_per_launch": f_roof,
                         "executed_flops_per_launch": f_exec,
                         "executed_frac": f_exec / (g_avg * 1e-3) / 1e12 / PEAK_TFLOPS[pname],
                         # The paper's operation count against this path's peak: comparable
                         # across kernels whose executed flops differ (padding, real
                         # products, work on the vector unit).
                         "alg_frac": f_alg / (g_avg * 1e-3) / 1e12 / PEAK_TFLOPS[pname],
                         "note": ("achieved = the paper-order algorithmic flops F_alg = 42 V n^2 + (22 + 8 n_mom) V "
                                  "n^3 per launch, on the FP64 issue rate the kernel's matrix and vector work share, "
                                  "/ mean event-timed duration of the contraction kernel; executed_frac counts the "
                                  "flops it executes (%s); step_frac uses the whole step" if paper_order else
                                  "achieved = flops one launch executes (%s) / mean event-timed duration of the "
                                  "contraction kernel; step_frac uses the whole step") % flops_note(pname, plan)
                                 + "; alg_frac = F_alg per launch / mean kernel duration / peak"},
        }
        print("# %-6s %.3f ms/block  %.1f blocks/s  contraction %.3f ms  reduce %.3f ms  w-image %.3f ms  "
              "MFMA %.1f TF (%.1f%% kernel, %.1f%% step)  err %s" % (
                  pname, step_ms, 1e3 / step_ms, g_avg, red_ms / max(1, launches), prep_ms / max(1, launches), ach,
                  100 * ach / PEAK_TFLOPS[pname], 100 * paths[pname]["roofline"]["step_frac"],
                  "%.2e" % err if err is not None else "-"), file=sys.stderr, flush=True)

    if args.calib_copy_mib > 0:
        nbytes = args.calib_copy_mib << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).uniform_()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print("# calibration: device copy and elementwise neg, each %d bytes read, %d bytes written"
              % (nbytes, nbytes), file=sys.stderr)

    # The headline is the paper's arithmetic (complex double, Sec. 4): the FP64
    # path; the split-precision paths are reported beside it.
    head = "fp64" if "fp64" in paths else next(iter(paths))
    hp = paths[head]
    rec = {
        "metric": METRIC,
        "value": hp["blocks_per_s"],
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hp["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic (seeded iid complex normal quark fields)",
        "config": {"workload": "headline-32: 32^3 sites, N_dil=32 (n1=n2=n3), 7 momenta {0, +-e_x, +-e_y, +-e_z}, "
                               "complex128 inputs, one timeslice per step",
                   "L": L, "n_dil": n, "n_mom": n_mom, "in_dtype": "c128", "blocks_per_step": 1},
        "tflops": {"gemm_count": hp["tflops_gemm_count"], "paper_count": hp["tflops_paper_count"]},
        "roofline": hp["roofline"],
        "paths": paths,
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(L, qs, mom, n * n)
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
