"""Benchmark: gradients/s of the batched complex64 adjoint path on one MI355X.

Workload (one step): quantum circuit learning at 20 qubits -- 64 data samples, each circuit RY(arcsin x_k)
on every qubit followed by 8 hardware-efficient layers (RY all, RZ all, CNOT ladder; 320 shared
parameters), observable Z_0, MSE loss against y = sin(pi x) + noise. One step = parameters into the
batch, forward pass of all 64 circuits (states, FP64 expectation reductions), loss on the device, and
the adjoint backward sweep that returns dL/dtheta: one full gradient. Inputs are synthetic and seeded.

Also reported: the same gradient by the parameter-shift rule on the same GPU (64 x 641 circuits through
the same batched engine, measured in full), by the plain per-circuit path (one global-memory pass per
gate, one circuit in flight; timed on a subset and extrapolated), the circuit-eval rate, the roofline
position of the dominant kernel (per-launch HIP events on the stream the kernels run on), and the CPU
oracle timed on the host on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--layers L] [--no-cpu] [--no-ps]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3   # published MI355X FP32 vector peak (256 CUs at 2.4 GHz)
TILE_KERNELS = ("rtile", "rtile_adj", "rtile_persist", "rtile_adj_persist", "tile", "tile_adj", "rtile_gen",
                "rtile_adj_gen")
SEED_PROFILE = 240603466 + 11


from paper_2406_03466_amd.profile_summary import kernel_source_hash  # noqa: E402


def pmc_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on the current
    kernel source."""
    p = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def summarize_launches(recs):
    per = {}
    for r in recs:
        k = per.setdefault(r["kernel"], {"launches": 0, "ms": 0.0, "bytes": 0, "flops": 0.0})
        k["launches"] += 1
        k["ms"] += r["ms"]
        k["bytes"] += r["bytes"]
        k["flops"] += r.get("flops", 0.0)
    for k in per.values():
        k["avg_ms"] = k["ms"] / k["launches"]
        k["avg_bytes"] = k["bytes"] / k["launches"]
        k["avg_flops"] = k["flops"] / k["launches"]
        k["gbs"] = (k["avg_bytes"] / 1e9) / (k["avg_ms"] / 1e3) if k["avg_ms"] > 0 else 0.0
        k["tflops"] = (k["avg_flops"] / 1e12) / (k["avg_ms"] / 1e3) if k["avg_ms"] > 0 else 0.0
    return per


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl_full, reps: int = 3):
    """The oracle (plain complex128 CPU simulator) on a bounded sample, timed twice: with one thread (the
    adjoint gradient of one sample) and with all host cores the box grants (one sample per thread, OpenMP
    over circuits); each `reps` times, mean and standard deviation, scaled to full gradients per second."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    out = {}
    for label, nth in (("one_thread", 1), ("all_cores", threads)):
        k = nth
        sub = wl_full.subset(range(k))
        e, _, _, _ = oracle.expectations(sub, nthreads=nth)
        up = 2.0 * (e - sub.extra["y"]) / wl_full.B
        ts = []
        for _ in range(reps):
            t0 = time.time()
            oracle.grad_adjoint(sub, up, nthreads=nth)
            ts.append(time.time() - t0)
        used = oracle.max_threads(nth)
        rates = [(k / wl_full.B) / t for t in ts]
        out[label] = {"gradients_per_s": float(np.mean(rates)), "sd": float(np.std(rates)), "threads": used,
                      "seconds_per_rep": [round(t, 3) for t in ts],
                      "sample": f"oracle adjoint gradient of {k} of the {wl_full.B} samples, scaled by {k}/{wl_full.B}"}
    a = out["all_cores"]
    return {"value": a["gradients_per_s"], "sd": a["sd"], "unit": "gradients/s", "cores": a["threads"],
            "kind": "oracle",
            "sample": f"oracle adjoint gradient (complex128) of {a['threads']} of the {wl_full.B} samples on "
                      f"{a['threads']} threads, mean of {reps}, scaled by {a['threads']}/{wl_full.B}",
            "one_thread": out["one_thread"], "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}


def copy_ceiling(torch, stream, reps: int = 10) -> dict:
    """A plain 1 GiB device-to-device copy (torch's copy kernel) timed with HIP events: the HBM rate a
    streaming kernel can reach on this GPU, beside the published 8 TB/s."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(reps):
        dst.copy_(src)
    ev[1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    nbytes = 2 * src.numel() * 8
    del src, dst
    return {"bytes_per_copy": nbytes, "ms": round(ms, 4), "gbs": round(nbytes / 1e9 / (ms / 1e3), 1),
            "frac_of_peak": round(nbytes / 1e9 / (ms / 1e3) / HBM_PEAK_GBS, 4)}


def stride_profile(qvpu, W, stream, sync, n: int) -> dict:
    """The stride engine alone on one n-qubit complex64 state: RY and RZ on every qubit (2n one-qubit
    gates, each one global-memory pass reading and writing the whole state), then the ZZ-chain
    expectation. Per-launch HIP events give each kernel's average time and algorithmic GB/s. Then the same
    forward call on the stride, LDS-tile and register-tile engines, each with its gate-equivalent GB/s."""
    gates = [W.gate(W.RY, q, -1, q) for q in range(n)] + [W.gate(W.RZ, q, -1, n + q) for q in range(n)]
    theta = np.random.default_rng(SEED_PROFILE).uniform(0, 2 * np.pi, 2 * n)
    zm = np.array([(1 << i) | (1 << (i + 1)) for i in range(n - 1)], np.uint64)
    wl = W.single(f"ryrz{n}", n, gates, theta, (np.zeros(n - 1, np.uint64), zm, np.ones(n - 1)))
    ctx = qvpu.Context(0, stream.cuda_stream, json.dumps({"engine": "stride", "graph": False,
                                                           "launch_events": True}))
    b = qvpu.Batch(ctx, wl, qvpu.QV_C64)
    b.expectations()
    sync()
    b.launch_log()
    for _ in range(3):
        b.expectations()
    sync()
    per = summarize_launches(b.launch_log())
    b.close()
    out = {"workload": f"{n} qubits complex64 ({(8 << n) / 2**30:.2f} GiB), {2 * n} one-qubit gates, "
                       f"{n - 1} ZZ terms; engine stride"}
    for k, v in per.items():
        out[k] = {"launches": v["launches"], "avg_ms": round(v["avg_ms"], 4),
                  "algorithmic_bytes_per_launch": int(v["avg_bytes"]), "gbs": round(v["gbs"], 1),
                  "frac_of_peak": round(v["gbs"] / HBM_PEAK_GBS, 4)}
    # the same forward call on each engine: what LDS tiles and register tiles buy over one pass per gate
    eng = {}
    for engine in ("stride", "lds", "tiled"):
        ctx = qvpu.Context(0, stream.cuda_stream, json.dumps({"engine": engine, "graph": True}))
        b = qvpu.Batch(ctx, wl, qvpu.QV_C64)
        sec = timed(lambda: b.expectations(), sync, 3)
        eng[engine] = {"forward_ms": round(sec * 1e3, 3), "passes": b.stats()["passes_per_circuit_max"],
                       "gate_equivalent": gate_equivalent(wl, 8, False, sec)}
        b.close()
    out["engines"] = eng
    return out


def unfused_bytes(wl, amp_bytes: int, adjoint: bool) -> int:
    """HBM bytes the plain per-gate method would move for one call over the batch: every gate one pass over
    the state (2S), every distinct x-mask of the observable one read (S); with adjoint, the seed lambda = H psi
    (read psi, write lambda: 2S) and every gate once more over psi and lambda (4S). Dividing by the measured
    time gives the "gate-equivalent" bandwidth, which shows what tiling and fusion buy over that method."""
    total = 0
    for b in range(wl.B):
        S = (1 << int(wl.n_qubits[b])) * amp_bytes
        G = int(wl.gate_offsets[b + 1] - wl.gate_offsets[b])
        groups = len(set(int(x) for x in wl.terms(b)[0])) if wl.term_offsets is not None else 0
        total += (2 * G + groups) * S
        if adjoint:
            total += (2 + 4 * G) * S
    return total


def gate_equivalent(wl, amp_bytes: int, adjoint: bool, seconds: float) -> dict:
    by = unfused_bytes(wl, amp_bytes, adjoint)
    gbs = by / seconds / 1e9
    return {"unfused_bytes": by, "gbs": round(gbs, 1), "times_hbm_peak": round(gbs / HBM_PEAK_GBS, 2)}


def timed(fn, stream_sync, reps: int = 1) -> float:
    """Seconds per call of fn after one untimed call (plans, buffers, graphs)."""
    fn()
    stream_sync()
    t0 = time.time()
    for _ in range(reps):
        fn()
    stream_sync()
    return (time.time() - t0) / reps


def other_workloads(qvpu, W, stream, sync, only=None, specialize="off", specialize_heavy=None) -> dict:
    """The other workload shapes, each on its own batch (created and freed here): circuit learning with 2
    and 4 layers (adjoint vs parameter-shift gradients/s), the 16-qubit VQE parameter-shift gradient (513
    circuits), 1024 uneven random circuits, MC-VQE-shaped batches at 16-22 qubits (adjoint and
    parameter-shift mean-energy gradients), DDCL-shaped circuits at 20-26 qubits (Jensen-Shannon loss
    gradients), and the 32-qubit 10-layer circuit (32 GiB complex64 state)
    forward and adjoint, with and without fused MFMA blocks."""
    out = {}

    # DDCL and the 32-qubit circuit have long passes: generating them costs minutes of compilation on a
    # machine with an empty cache, so the full benchmark can run them with another "specialize" setting
    heavy = specialize if specialize_heavy is None else specialize_heavy
    t_start = time.time()

    def done(key):   # progress on stderr while the one JSON line waits
        print(f"# {key} done at {time.time() - t_start:.0f} s", file=sys.stderr, flush=True)

    def ctx(**o):
        o.setdefault("graph", True)
        o.setdefault("specialize", specialize)
        return qvpu.Context(0, stream.cuda_stream, json.dumps(o))

    # circuit learning at 20 qubits with 2 and 4 layers: adjoint gradient vs parameter-shift, same engine
    for layers in ((2, 4) if only in (None, "qcl") else ()):
        wl = W.config3(layers)
        b = qvpu.Batch(ctx(fusion="8"), wl, qvpu.QV_C64)
        e, _ = b.expectations(want_terms=False)
        up = 2.0 * (e - wl.extra["y"]) / wl.B

        def grad(method):
            b.expectations(want_terms=False)
            b.gradient(method, upstream=up)

        s_ad = timed(lambda: grad(qvpu.QV_ADJOINT), sync, 3)
        s_ps = timed(lambda: b.gradient(qvpu.QV_PARAM_SHIFT, upstream=up), sync, 1)
        out[f"qcl20_L{layers}_S64"] = {"adjoint_gradients_per_s": round(1.0 / s_ad, 3),
                                       "param_shift_gradients_per_s": round(1.0 / s_ps, 4),
                                       "speedup": round(s_ps / s_ad, 1),
                                       "param_shift_circuits": wl.B * (2 * wl.n_grad() + 1)}
        done(f"qcl20_L{layers}_S64")
        b.close()
    # the benchmark workload in complex128 (FP64 throughout; register tiles of 2^12 amplitudes), with the
    # general tile kernels and with generated adjoint passes where they time faster
    if only in (None, "qcl"):
        wl = W.config3(8)
        rec = {}
        for spec in ("off", "auto"):
            b = qvpu.Batch(ctx(fusion="off", specialize=spec), wl, qvpu.QV_C128)
            e, _ = b.expectations(want_terms=False)
            up = 2.0 * (e - wl.extra["y"]) / wl.B

            def grad128():
                b.expectations(want_terms=False)
                b.gradient(qvpu.QV_ADJOINT, upstream=up)

            s_ad = timed(grad128, sync, 3)
            key = "" if spec == "off" else "_specialize_auto"
            rec["adjoint_gradients_per_s" + key] = round(1.0 / s_ad, 3)
            rec["ms" + key] = round(s_ad * 1e3, 3)
            b.close()
        out["qcl20_L8_S64_c128"] = rec
        done("qcl20_L8_S64_c128")
    # the 16-qubit VQE parameter-shift gradient (513 circuits) and 1024 uneven random circuits, each with
    # one launch per pass level and with every sweep in one persistent launch
    wl = W.config2()
    for prec, name in ([(qvpu.QV_C64, "c64"), (qvpu.QV_C128, "c128")] if only in (None, "hea16") else []):
        rec = {"circuits": 513}
        for launch in ("levels", "persistent"):
            b = qvpu.Batch(ctx(launch=launch), wl, prec)
            s = timed(lambda: b.gradient(qvpu.QV_PARAM_SHIFT), sync, 3)
            key = "" if launch == "levels" else "_persistent"
            rec["circuit_evals_per_s" + key] = round(513 / s, 1)
            rec["gradient_ms" + key] = round(s * 1e3, 3)
            b.close()
        out[f"hea16_L8_T100_param_shift_{name}"] = rec
        done(f"hea16_L8_T100_param_shift_{name}")
    if only in (None, "random1024"):
        wl = W.config4()
        rec = {"circuits": wl.B}
        for launch in ("levels", "persistent"):
            b = qvpu.Batch(ctx(launch=launch), wl, qvpu.QV_C64)
            s = timed(lambda: b.expectations(), sync, 3)
            key = "" if launch == "levels" else "_persistent"
            rec["circuit_evals_per_s" + key] = round(wl.B / s, 1)
            rec["ms" + key] = round(s * 1e3, 3)
            if launch == "levels":
                rec["gate_equivalent"] = gate_equivalent(wl, 8, False, s)
            b.close()
        out["random1024_expectations_c64"] = rec
        done("random1024_expectations_c64")
    # MC-VQE-shaped batches at Table 1's sizes: one circuit per CIS state, mean-energy gradient
    for nq in ((16, 18, 20, 22) if only in (None, "mcvqe") else ()):
        wl = W.mcvqe(nq)
        up = np.full(wl.B, 1.0 / wl.B)
        b = qvpu.Batch(ctx(), wl, qvpu.QV_C64)
        s_ad = timed(lambda: b.gradient(qvpu.QV_ADJOINT, upstream=up), sync, 3)
        s_ps = timed(lambda: b.gradient(qvpu.QV_PARAM_SHIFT, upstream=up), sync, 1)
        nh, P = wl.extra["n_hamiltonian_terms"], wl.n_grad()
        out[f"mcvqe{nq}_S{wl.B}_c64"] = {"adjoint_gradient_ms": round(s_ad * 1e3, 3),
                                        "param_shift_gradient_ms": round(s_ps * 1e3, 3),
                                        "param_shift_circuits": wl.B * (2 * P + 1),
                                        "param_shift_circuit_evals_per_s": round(wl.B * (2 * P + 1) / s_ps, 1),
                                        "terms": nh, "params": P, "per_state_per_term_circuits": 2 * nh * P}
        done(f"mcvqe{nq}_S{wl.B}_c64")
        b.close()
    # DDCL-shaped circuits at Table 2's sizes (10 layers, 60 N_q parameters): Jensen-Shannon loss gradient
    for nq in ((20, 22, 24, 26) if only in (None, "ddcl") else ()):
        wl = W.ddcl(nq, 10)
        t = wl.extra["target"]
        b = qvpu.Batch(ctx(specialize=heavy), wl, qvpu.QV_C64)
        s_ad = timed(lambda: b.js_gradient(t, qvpu.QV_ADJOINT), sync, 3)
        rec = {"adjoint_gradient_ms": round(s_ad * 1e3, 3), "params": wl.n_grad(),
               "param_shift_circuits": 2 * wl.n_grad() + 1}
        if nq <= 22:
            s_ps = timed(lambda: b.js_gradient(t, qvpu.QV_PARAM_SHIFT), sync, 1)
            rec["param_shift_gradient_ms"] = round(s_ps * 1e3, 2)
            rec["param_shift_circuit_evals_per_s"] = round((2 * wl.n_grad() + 1) / s_ps, 1)
            rec["param_shift_measured"] = "full gradient"
        b.close()
        if nq > 22:
            # the same circuit with only its first K angles trainable (the rest fixed at their values):
            # 2K + 1 circuits timed, the full gradient's 2 N_theta + 1 extrapolated per circuit
            K = 64
            g = wl.gates.copy()
            keep = g["param"] < K
            g["angle"][~keep] = wl.theta[g["param"][~keep]]
            g["param"][~keep] = -1
            sub = W.Workload(wl.name + f"[{K} params]", wl.n_qubits, wl.gate_offsets, g, np.array([K], np.int32),
                             False, wl.theta[:K].copy(), wl.term_offsets, wl.xmask, wl.zmask, wl.coeff, False,
                             dict(wl.extra))
            b = qvpu.Batch(ctx(specialize=heavy), sub, qvpu.QV_C64)
            s_ps = timed(lambda: b.js_gradient(t, qvpu.QV_PARAM_SHIFT), sync, 1)
            per = s_ps / (2 * K + 1)
            rec["param_shift_gradient_ms"] = round(per * (2 * wl.n_grad() + 1) * 1e3, 1)
            rec["param_shift_circuit_evals_per_s"] = round(1.0 / per, 1)
            rec["param_shift_measured"] = f"extrapolated: {2 * K + 1} circuits timed ({s_ps * 1e3:.1f} ms)"
            b.close()
        out[f"ddcl{nq}_L10_c64"] = rec
        done(f"ddcl{nq}_L10_c64")
    wl = W.config5() if only in (None, "hea32") else None
    for fusion in (["off", "8"] if wl is not None else []):
        b = qvpu.Batch(ctx(fusion=fusion, tile_qubits=13, specialize=heavy), wl, qvpu.QV_C64)
        sf = timed(lambda: b.expectations(), sync, 1)
        sg = timed(lambda: b.gradient(qvpu.QV_ADJOINT), sync, 1)
        st = b.stats()
        out[f"hea32_L10_c64_fusion_{fusion}"] = {"forward_ms": round(sf * 1e3, 2), "gradient_ms": round(sg * 1e3, 2),
                                                  "passes": st["passes_per_circuit_max"],
                                                  "gate_equivalent_forward": gate_equivalent(wl, 8, False, sf),
                                                  "gate_equivalent_gradient": gate_equivalent(wl, 8, True, sg)}
        done(f"hea32_L10_c64_fusion_{fusion}")
        b.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--layers", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ps", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the other workload shapes")
    ap.add_argument("--only", choices=["qcl", "hea16", "random1024", "hea32", "mcvqe", "ddcl", "stride"],
                    help="run only this one of the other workload shapes and print its figures")
    ap.add_argument("--qubits", type=int, default=26, help="state size of --only stride")
    ap.add_argument("--tile-qubits", type=int, default=0)
    ap.add_argument("--engine", default="tiled", choices=["tiled", "lds", "stride"])
    ap.add_argument("--contig", type=int, default=0)
    ap.add_argument("--launch", default="levels", choices=["levels", "persistent"])
    ap.add_argument("--fusion", default="auto",
                    help='fused 4-qubit MFMA blocks in forward passes: "off", "on", "auto" (the autotuner picks '
                         'the minimum run) or a minimum run length')
    ap.add_argument("--specialize", default="auto", choices=["off", "adjoint", "on", "auto"],
                    help="register-tiled levels run kernels generated for their pass (adjoint sweeps, or both)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--levels", action="store_true", help="print per-launch times of one step")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: the whole batch is one GPU's share; "
                                   "run with --gpus 1"}))
        sys.exit(2)

    import torch
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8}), flush=True)
        return
    from paper_2406_03466_amd import qvpu
    from paper_2406_03466_amd import workloads as W
    from paper_2406_03466_amd.autograd import expectation
    if args.only:
        st = torch.cuda.current_stream(torch.device("cuda:0"))
        if args.only == "stride":
            out = stride_profile(qvpu, W, st, torch.cuda.synchronize, args.qubits)
            out["copy_ceiling"] = copy_ceiling(torch, st)
            print(json.dumps(out), flush=True)
            return
        print(json.dumps(other_workloads(qvpu, W, st, torch.cuda.synchronize, args.only, args.specialize)),
              flush=True)
        return

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = W.config3(args.layers)
    stream = torch.cuda.current_stream(dev)
    opts = {"graph": False, "launch_events": True, "engine": args.engine, "launch": args.launch,
            "fusion": args.fusion, "specialize": args.specialize}
    if args.tile_qubits:
        opts["tile_qubits"] = args.tile_qubits
    if args.contig:
        opts["contig_qubits"] = args.contig
    if not args.tile_qubits and not args.contig:
        opts["autotune"] = "search"
    ctx = qvpu.Context(0, stream.cuda_stream, json.dumps(opts))
    batch = qvpu.Batch(ctx, wl, qvpu.QV_C64)
    theta = torch.tensor(wl.theta, dtype=torch.float64, device=dev, requires_grad=True)
    y = torch.tensor(wl.extra["y"], dtype=torch.float64, device=dev)

    def step():
        theta.grad = None
        f = expectation(theta, batch)
        loss = torch.mean((f - y) ** 2)
        loss.backward()
        return loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    recs = []
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    batch.launch_log()  # drop the warm-up records
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t_start.record(stream)
    marks[0].record(stream)
    for i in range(args.steps):
        step()
        marks[i + 1].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    step_ms = [marks[i].elapsed_time(marks[i + 1]) for i in range(args.steps)]
    recs = batch.launch_log()
    tuned = batch.stats()
    if args.levels:
        per_step = len(recs) // max(1, args.steps)
        for r in recs[:per_step]:
            print(f"# {r['kernel']:12s} level {r['level']:3d} {r['ms']:9.4f} ms {r['bytes'] / 1e9:8.3f} GB", flush=True)
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    grads_per_s = 1000.0 / ms_step
    per = summarize_launches(recs)
    dom = max(per, key=lambda k: per[k]["ms"])
    d = per[dom]
    achieved = d["gbs"]
    kernel_sym = {"tile_adj": "k_tile<float,true>", "tile": "k_tile<float,false>",
                  "rtile_adj": "k_rtile_adj<float,4,512>", "rtile": "k_rtile_fwd<float,4,512>",
                  "rtile_adj_persist": "k_rtile_adj_persist<float,4,512>",
                  "rtile_persist": "k_rtile_fwd_persist<float,4,512>",
                  "rtile_adj_gen": "qv_gen_adj (generated adjoint tile pass, complex64)",
                  "rtile_gen": "qv_gen_fwd (generated forward tile pass, complex64)"}.get(dom, dom)
    workload_tag = f"qcl20_L{args.layers}"
    traffic = pmc_traffic(dom, workload_tag)
    if dom in TILE_KERNELS:
        # register/LDS tile passes run tens of gates per HBM round trip: bound by vector ALU issue
        roofline = {"bound": "alu", "achieved": round(d["tflops"], 2), "peak": FP32_VECTOR_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(d["tflops"] / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": traffic,
                    "kernel": kernel_sym, "launches": d["launches"], "avg_launch_ms": round(d["avg_ms"], 4),
                    "algorithmic_flops_per_launch": d["avg_flops"],
                    "algorithmic_bytes_per_launch": int(d["avg_bytes"]),
                    "hbm_gbs": round(achieved, 1), "hbm_frac": round(achieved / HBM_PEAK_GBS, 4)}
    else:
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel_sym,
                    "launches": d["launches"], "avg_launch_ms": round(d["avg_ms"], 4),
                    "algorithmic_bytes_per_launch": int(d["avg_bytes"])}
    # fused 4-qubit blocks of the forward passes run on MFMA (a 32 x 32 real product per 16 amplitudes,
    # 128 flops per amplitude per block); their flops are reported apart from the gates' algorithmic flops
    fuse_min = tuned["fuse_min_run"]   # the run length the batch uses (chosen by the autotuner under "auto")
    n_fused = 0
    if fuse_min and args.engine == "tiled":
        n_fused = sum(p["n_fused"] for p in qvpu.plan_circuit(20, wl.circuit(0), tuned["tile_qubits"], qvpu.QV_C64,
                                                               0, fuse_min=fuse_min))
    fused = {"blocks_per_circuit": n_fused, "mfma_flops_per_forward": n_fused * 128.0 * (1 << 20) * wl.B}
    # forward-only circuit evals/s (the 64 circuits of one forward pass)
    fwd_ms = sum(r["ms"] for r in recs if r["kernel"] in ("matrices", "fuse", "init", "tile", "rtile",
                                                          "rtile_persist", "rtile_gen", "stride", "expect",
                                                          "finalize")) / args.steps
    circuit_evals_per_s = wl.B / (fwd_ms / 1e3)

    extra = {}
    if not args.no_ps:
        # parameter-shift gradient through the same batched tiled engine, measured in full
        ctx_ps = qvpu.Context(0, stream.cuda_stream, json.dumps({"graph": False, "fusion": args.fusion,
                                                                 "specialize": args.specialize}))
        b_ps = qvpu.Batch(ctx_ps, wl, qvpu.QV_C64)
        with torch.no_grad():
            f = expectation(theta.detach(), batch)
            up = (2.0 * (f - y) / wl.B).contiguous()
        g_buf = torch.empty(wl.n_grad(), dtype=torch.float64, device=dev)
        b_ps.gradient(qvpu.QV_PARAM_SHIFT, upstream=up, grad=g_buf)  # warm-up (plans, buffers)
        torch.cuda.synchronize()
        t0 = time.time()
        b_ps.gradient(qvpu.QV_PARAM_SHIFT, upstream=up, grad=g_buf)
        torch.cuda.synchronize()
        ps_s = time.time() - t0
        g_ad = theta.grad.detach().clone() if theta.grad is not None else None
        n_ps_circ = wl.B * (2 * int(np.sum(wl.circuit(0)["param"] >= 0)) + 1)
        extra["param_shift_tiled"] = {"gradients_per_s": 1.0 / ps_s, "seconds": ps_s, "circuits": n_ps_circ,
                                      "measured": "full gradient"}
        if g_ad is not None:
            scale = float(torch.sum(torch.abs(up)).item())
            extra["adjoint_vs_param_shift_max_abs_diff_over_scale"] = float(
                torch.max(torch.abs(g_ad - g_buf)).item() / max(scale, 1e-300))
        del b_ps, ctx_ps
        # plain per-circuit path: one global-memory pass per gate, one circuit in flight, on a subset
        sub = wl.subset([0])
        ctx_pl = qvpu.Context(0, stream.cuda_stream,
                              json.dumps({"graph": False, "engine": "stride", "n-virtual-qpus": 1}))
        b_pl = qvpu.Batch(ctx_pl, sub, qvpu.QV_C64)
        b_pl.expectations(want_terms=False)
        torch.cuda.synchronize()
        t0 = time.time()
        b_pl.expectations(want_terms=False)
        torch.cuda.synchronize()
        one_circ_s = time.time() - t0
        ps_plain_s = one_circ_s * n_ps_circ
        extra["param_shift_plain"] = {"gradients_per_s": 1.0 / ps_plain_s, "seconds": ps_plain_s,
                                      "circuits": n_ps_circ,
                                      "measured": f"extrapolated: one circuit timed ({one_circ_s * 1e3:.2f} ms) "
                                                  f"x {n_ps_circ} circuits"}
        extra["adjoint_speedup_vs_param_shift_tiled"] = grads_per_s * ps_s
        extra["adjoint_speedup_vs_param_shift_plain"] = grads_per_s * ps_plain_s
        del b_pl, ctx_pl

    out = {
        "metric": "gradients/s (adjoint vs param-shift) at 20q; circuit evals/s; HBM GB/s vs peak",
        "value": round(grads_per_s, 3),
        "unit": "gradients/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_sd": round(float(np.std(step_ms)), 4),
        "gradient_s_mean_sd": [round(float(np.mean(step_ms)) / 1e3, 6), round(float(np.std(step_ms)) / 1e3, 6)],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic (seeded; the paper's datasets are not published)",
        "config": {"workload": f"qcl20_L{args.layers}_S64: quantum circuit learning, 20 qubits, 64 samples, "
                               f"RY(arcsin x) encoding + {args.layers} HEA layers ({wl.n_grad()} params), "
                               f"<Z_0>, MSE loss, adjoint gradient, complex64 with FP64 reductions",
                   "qubits": 20, "layers": args.layers, "samples": 64, "params": wl.n_grad(),
                   "precision": "c64", "engine": args.engine, "tile_qubits": tuned["tile_qubits"],
                   "contig_qubits": tuned["contig_qubits"], "passes": tuned["passes_per_circuit_max"],
                   "fuse_min_run": tuned["fuse_min_run"],
                   "autotuned": not (args.tile_qubits or args.contig), "launch": args.launch,
                   "fusion": args.fusion, "specialize": args.specialize},
        "roofline": roofline,
        "gate_equivalent": gate_equivalent(wl, 8, True, ms_step / 1e3),
        "fused_blocks": fused,
        "circuit_evals_per_s": round(circuit_evals_per_s, 1),
        "kernels": {k: {"launches": v["launches"], "avg_ms": round(v["avg_ms"], 4), "gbs": round(v["gbs"], 1),
                        "tflops": round(v["tflops"], 2)} for k, v in per.items()},
        "kernel_source_hash": kernel_source_hash(),
    }
    out.update(extra)
    out["copy_ceiling"] = copy_ceiling(torch, stream)
    if not args.no_extras:
        out["other_workloads"] = other_workloads(qvpu, W, stream, torch.cuda.synchronize, None, args.specialize, "off")
        out["other_workloads"]["stride26_c64"] = stride_profile(qvpu, W, stream, torch.cuda.synchronize, 26)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
