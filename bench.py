"""Benchmark: density matrices per second for the learned Fermi-operator expansion on one GPU.

A step is one full fe_expand_density call on a resident Hamiltonian: Gershgorin bounds, rescale,
all L layers (split-precision MFMA products with the fused epilogue) and the FP64 traces.

Workload: 16^3 periodic Anderson lattice (N = 4096), hopping -1, on-site disorder U[-1, 1],
kT = 0.05, mu = 0. The step selects the model from the bank of trained coefficient sets (fewest
layers whose region of validity holds the matrix's beta' and mu', Sec. on the region of validity
by layer count; for this lattice beta' = 280 and mu' = 1/2 select the 20-layer beta0 = 300,
mu0 = 1/2 model) and then expands; the paper's 26-layer (beta0 = 1500, mu0 = 1/3) model is timed
beside it, and so are the entropy expansion (the trained entropy model selected the same way)
and the final correction layer.

Prints one JSON line with the throughput, the roofline of the layer kernel (each layer launch
timed live with HIP events the library records on the launch stream), the error against the CPU
FP64 eigendecomposition oracle, the baselines on the same GPU (plain FP64 recursion with vendor
DGEMM, FP64 eigensolver) and the oracle timed on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("density matrices/s and TFLOP/s vs FP64 recursion & eigensolver at "
          "‖ΔD‖_F/N≤1e-5")
PEAK_TFLOPS = {"fp16x2": 2500.0, "bf16x2": 2500.0, "bf16x3": 2500.0, "fp32": 157.3, "fp64": 78.6}
HBM_GBS = 8000.0
# The model bank: trained families at mu0 = 1/3, 0.4 and 1/2, each fitted to <= 1e-7 max error
# (each matrix runs the fewest layers whose region of validity holds its (beta', mu'))
BANK = ["mlsp2_L20_b300_mu1third", "mlsp2_L22_b600_mu1third", "mlsp2_L26_b1500_mu1third",
        "mlsp2_L40_b1e4_mu1third",
        "mlsp2_L18_b150_mu0p4", "mlsp2_L19_b200_mu0p4", "mlsp2_L20_b300_mu0p4",
        "mlsp2_L22_b600_mu0p4", "mlsp2_L26_b1500_mu0p4",
        "mlsp2_L18_b150_mu0p5", "mlsp2_L19_b200_mu0p5", "mlsp2_L20_b300_mu0p5",
        "mlsp2_L22_b600_mu0p5", "mlsp2_L24_b1500_mu0p5", "mlsp2_L27_b3000_mu0p5",
        "mlsp2_L29_b4000_mu0p5", "mlsp2_L36_b1e4_mu0p5"]
# trained entropy models (theta_entropy, Sec. III.B), selected per matrix by the same rule
ENTROPY_BANK = ["entropy_L26_b40_mu1third", "entropy_L26_b1500_mu1third", "entropy_L40_b1e4_mu1third"]
LARGE_ORACLE = os.path.join(ROOT, "tests", "golden", "large16384_oracle.npz")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--prec", default="fp16x2", choices=["fp16x2", "bf16x2", "bf16x3"],
                   help="bf16x3 (three-part BF16 split, six products): batch1024 only")
    p.add_argument("--batch-launch", default="auto", choices=["auto", "queue", "layers"],
                   help="batch1024: the plan tuner's choice (default), every layer in one queue "
                        "launch, or one grouped launch per layer")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-gpu-baselines", action="store_true")
    p.add_argument("--profile", action="store_true", help="only the timed steps (for rocprofv3)")
    p.add_argument("--workload", default="anderson4096",
                   choices=["anderson4096", "small128", "batch1024", "large16384", "filling4096",
                            "variants4096", "sweep", "train"],
                   help="anderson4096: the headline line (default); small128: one N = 128 FP64 "
                        "solve, 30 layers; batch1024: 1024 uneven "
                        "matrices in one captured plan; large16384: one N = 16384 solve, "
                        "density and entropy; filling4096: Newton mu at half filling; "
                        "variants4096: Skip-SP2 / Max-SP2; sweep: ms per D vs N; train: the "
                        "coefficient fit and the matrix forward/backward")
    p.add_argument("--model", default="bank",
                   help="anderson4096: 'bank' (select per matrix, default) or one model name")
    p.add_argument("--vendor-gemm", action="store_true",
                   help="only the vendor FP16 GEMM (torch.matmul) on a plain 4096^3 product, 20 "
                        "times (the reference for the layer kernel's MFMA counters)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only a plain 1 GiB device-to-device copy, three times (the reference for "
                        "scaling the HBM byte counters)")
    return p.parse_args()


def norm2_sym(E, torch, dev):
    """Spectral norm of a symmetric error matrix (the paper's norm): max |eigenvalue|, FP64 on the
    GPU (E: numpy array or tensor)."""
    T = E if isinstance(E, torch.Tensor) else torch.from_numpy(E)
    return float(torch.linalg.eigvalsh(T.to(device=dev, dtype=torch.float64)).abs().max().item())


def timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps     # ms per call


KERNEL_SOURCES = ("fe_api.hip", "fe_internal.h", "k_layer_split.hip", "split_common.h")
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "k_layer_split_counters_anderson4096.md")
SQ_SUMMARY = os.path.join(ROOT, "profiles", "k_layer_split_sq_counters_anderson4096.md")
TRACE_SUMMARY = os.path.join(ROOT, "profiles", "k_layer_split_anderson4096_fp16x2.md")


def _profile_record(path, tag):
    """The JSON record after `tag:` in a committed profile summary, or None if it is missing or
    the layer kernel's sources changed since the counters were taken (SHA-256 over them)."""
    import hashlib
    try:
        line = next(l for l in open(path) if l.startswith(tag + ":"))
        rec = json.loads(line.split(":", 1)[1])
    except (OSError, StopIteration, ValueError):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_08523_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return rec if h.hexdigest() == rec.get("source_sha256") else None


def measured_traffic():
    """HBM bytes per layer launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary
    (copy-calibrated), or None if the layer kernel's sources changed since it was taken."""
    rec = _profile_record(COUNTER_SUMMARY, "traffic_json")
    return rec["bytes_per_launch"] if rec else None


def measured_profile():
    """The rocprofv3 kernel-trace average of the layer kernel and the event figure of the same
    session, from the committed summary (None if the layer kernel's sources changed since)."""
    rec = _profile_record(TRACE_SUMMARY, "trace_json")
    return rec


def measured_pipe_busy():
    """Clock and MFMA-pipe occupancy of the layer kernel from the committed SQ-counter summary
    (None if stale)."""
    rec = _profile_record(SQ_SUMMARY, "sq_json")
    return {k: rec[k] for k in ("clock_ghz", "mfma_pipe_busy", "vendor_gemm_mfma_pipe_busy")} if rec else None


def layer_event_ms(api, expand, torch, reps=10):
    """Duration of each layer launch of the split path, from HIP events the library records on the
    launch stream around every layer launch (fe_debug_layer_events), over `reps` expansions."""
    expand()
    torch.cuda.synchronize()
    api.layer_events(True)
    per = []
    try:
        for _ in range(reps):
            expand()
            per.extend(api.layer_events_read().tolist())
    finally:
        api.layer_events(False)
    per.sort()
    return {"mean": sum(per) / len(per), "median": per[len(per) // 2], "launches": len(per)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the expansion of one matrix is not sharded across GPUs in this build)", file=sys.stderr)
        sys.exit(2)
    if args.prec == "bf16x3" and args.workload != "batch1024":
        print("--prec bf16x3 is measured on the batch1024 workload only", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2605_08523_amd import api, models, workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        x = torch.ones(256 * 2**20, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print("copy calibration done: 3 copies of 1 GiB", flush=True)
        return
    if args.vendor_gemm:
        n = 4096
        ga = torch.randn(n, n, device=dev, dtype=torch.float16)
        gb = torch.randn(n, n, device=dev, dtype=torch.float16).t().contiguous()
        ms = timed(lambda: ga @ gb, 20, 3, torch)
        print(f"vendor fp16 gemm {n}^3: {ms * 1e3:.1f} us, {2.0 * n ** 3 / ms / 1e9:.1f} TFLOP/s",
              flush=True)
        return
    if args.workload == "batch1024":
        return bench_batch(args, torch, api, models, workloads, dev)
    if args.workload == "large16384":
        return bench_large(args, torch, api, models, workloads, dev)
    if args.workload == "filling4096":
        return bench_filling(args, torch, api, models, workloads, dev)
    if args.workload == "variants4096":
        return bench_variants(args, torch, api, models, workloads, dev)
    if args.workload == "sweep":
        return bench_sweep(args, torch, api, models, workloads, dev)
    if args.workload == "train":
        return bench_train(args, torch, api, models, workloads, dev)
    if args.workload == "small128":
        return bench_small(args, torch, api, models, workloads, dev)
    c = workloads.config_anderson_4096()
    H = c["H"]
    n = H.shape[0]
    Hd = torch.from_numpy(H).to(dev)
    mu, kT = c["mu"], c["kT"]
    ws = api.Workspace(n)
    D = torch.empty((n, n), dtype=torch.float32, device=dev)
    if args.model == "bank":
        bank = [models.load(x) for x in BANK]
        bank_refs = [api.make_model(x.theta, x.beta0, x.mu0) for x in bank]
        m = bank[api.select_model(Hd, mu, kT, bank_refs, ws=ws)]
    else:
        bank = None
        m = models.load(args.model)
    mref = api.make_model(m.theta, m.beta0, m.mu0)
    m1 = api.make_model(m.theta[-1:], m.beta0, m.mu0)      # one layer: prologue + one layer
    # tile shape / schedule chosen by the autotuner on this input (recorded for the timed runs)
    tuned = api.autotune_input(Hd, mu, kT, mref, prec=args.prec, ws=ws) if not args.profile else None

    def expand():
        api.expand_density(Hd, mu, kT, mref, prec=args.prec, out=D, ws=ws)

    def step():
        if bank is not None:
            k = api.select_model(Hd, mu, kT, bank_refs, ws=ws)
            api.expand_density(Hd, mu, kT, bank_refs[k], prec=args.prec, out=D, ws=ws)
        else:
            expand()

    def step1():
        api.expand_density(Hd, mu, kT, m1, prec=args.prec, out=D, ws=ws)

    # correctness of the timed configuration first (info synchronizes)
    _, trD, trD2, info = api.expand_density(Hd, mu, kT, mref, prec=args.prec, out=D, ws=ws,
                                            want_info=True)
    if args.profile:
        for _ in range(args.warmup + args.steps):
            step()
        torch.cuda.synchronize()
        lay = layer_event_ms(api, expand, torch)
        print(f"profile run done; layer launch (HIP events, this process): mean {lay['mean']:.4f} "
              f"ms over {lay['launches']} launches, model {m.name}", flush=True)
        return

    ms = timed(step, args.steps, args.warmup, torch)
    # per-step distribution: events around each step of a second pass
    per = []
    for _ in range(max(20, args.steps)):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        step()
        e1.record()
        per.append((e0, e1))
    torch.cuda.synchronize()
    per_ms = sorted(a.elapsed_time(b) for a, b in per)
    ms_expand = timed(expand, args.steps, args.warmup, torch) if bank is not None else ms
    ms1 = timed(step1, args.steps, args.warmup, torch)
    L = m.L
    layer_ms_diff = (ms_expand - ms1) / (L - 1)
    lay = layer_event_ms(api, expand, torch)
    layer_ms = lay["mean"]
    flop_layer = 2.0 * n ** 3                         # algorithmic X^2 of one layer
    # executed MFMA work: three products on the upper tiles of the schedule the tuner chose
    sched = api.autotune_lookup(n, prec=args.prec, ws=ws)
    tile = 256 if sched == "sk256" else 128
    T = -(-n // tile)
    np_ = T * tile
    exec_flop_layer = 3 * 2.0 * (T * (T + 1) // 2) * tile * tile * np_   # three MFMA products, upper tiles
    achieved = flop_layer / (layer_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.prec]
    value = 1000.0 / ms
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "density matrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16" if args.prec == "fp16x2" else "bf16",
        "precision": f"{args.prec}: 16-bit hi/lo split, 3 MFMA products, fp32 accumulate; fp64 bounds, rescale and traces",
        "data": "synthetic",
        "config": {"workload": "anderson_cubic_16x16x16_periodic_N4096_t-1_W1_kT0.05_mu0",
                   "N": n, "layers": L, "coefficients": m.name, "seed": c["seed"],
                   "model_selection": ("fewest layers valid for (beta', mu') among " + ", ".join(BANK)
                                       + "; selection (bounds pass + read-back) inside the step")
                   if bank is not None else "fixed"},
        "tflops_algorithmic": L * flop_layer / (ms * 1e-3) / 1e12,
        "roofline": {
            "kernel": "k_layer_split (one layer: split MFMA X^2 + fused epilogue)",
            "bound": "mfma",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": measured_traffic(),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "layer_ms": layer_ms,
            "executed_mfma_tflops": exec_flop_layer / (layer_ms * 1e-3) / 1e12,
            "executed_frac": exec_flop_layer / (layer_ms * 1e-3) / 1e12 / peak,
            "sq_counters": measured_pipe_busy(),
            "schedule": sched,
            "method": (f"HIP events recorded by the library on the launch stream around each of the "
                       f"{L} layer launches of an expansion, mean over {lay['launches']} launches "
                       f"(median {lay['median']:.4f} ms); by differencing expansions, "
                       f"(t(L={L}) - t(L=1)) / {L - 1} = {layer_ms_diff:.4f} ms"),
            "layer_ms_by_differencing": layer_ms_diff,
            "profile": measured_profile(),
        },
        "prologue_plus_one_layer_ms": ms1,
        "autotune": tuned,
        "ms_per_step_median": per_ms[len(per_ms) // 2],
        "ms_per_step_p90": per_ms[int(0.9 * (len(per_ms) - 1))],
    }
    # the whole single-matrix path of Alg. 2: density and entropy, the entropy with the trained
    # entropy coefficients (theta_entropy) selected for this matrix like the density model
    ebank = [models.load(x) for x in ENTROPY_BANK]
    ebank_refs = [api.make_model(x.theta, x.beta0, x.mu0) for x in ebank]
    ke = api.select_model(Hd, mu, kT, ebank_refs, ws=ws)
    ment, mentref = ebank[ke], ebank_refs[ke]
    ms_ds = timed(lambda: (step(), api.expand_entropy(Hd, mu, kT, mentref, ment.alpha,
                                                      prec=args.prec, ws=ws)),
                  args.steps, args.warmup, torch)
    out["step_with_entropy"] = {"ms": ms_ds, "per_s": 1000.0 / ms_ds,
                                "entropy_model": ment.name,
                                "what": "model selection + density + entropy expansion (theta_entropy)"}
    if bank is not None:
        out["expand_only_ms"] = ms_expand
        m26 = models.load("mlsp2_L26_b1500_mu1third")
        r26 = api.make_model(m26.theta, m26.beta0, m26.mu0)
        ms26 = timed(lambda: api.expand_density(Hd, mu, kT, r26, prec=args.prec, out=D, ws=ws),
                     args.steps, args.warmup, torch)
        out["fixed_model_L26"] = {"coefficients": m26.name, "ms_per_step": ms26,
                                  "value": 1000.0 / ms26}
    # the squared-affine layer form (opt-in, FE_FORM=affine): same step, its own error below
    Daff = None
    if args.prec == "fp16x2":
        os.environ["FE_FORM"] = "affine"
        try:
            ms_aff = timed(step, args.steps, args.warmup, torch)
            api.expand_density(Hd, mu, kT, mref, prec=args.prec, out=D, ws=ws)
            torch.cuda.synchronize()
            Daff = D.double().cpu().numpy()
        finally:
            del os.environ["FE_FORM"]
        out["affine_form"] = {"ms_per_step": ms_aff, "value": 1000.0 / ms_aff,
                              "what": "FE_FORM=affine: operand = shifted state, no FP32 state "
                                      "traffic in the epilogue"}
    # the final correction layer (last product by FP32 MFMA, FP64 epilogue, float64 D), opt-in
    D64 = torch.empty((n, n), dtype=torch.float64, device=dev)
    ms_corr = timed(lambda: api.expand_density(Hd, mu, kT, mref, prec=args.prec, out=D64, ws=ws,
                                               final_correction=True), args.steps, args.warmup,
                    torch)
    api.expand_density(Hd, mu, kT, mref, prec=args.prec, out=D64, ws=ws, final_correction=True)
    torch.cuda.synchronize()
    Dcorr = D64.cpu().numpy()
    del D64
    out["final_correction"] = {"ms_expand": ms_corr, "ms_expand_without": ms_expand,
                               "what": "final_correction=1: last layer X^2 by FP32 MFMA from the "
                                       "FP32 state, D = A + d X + (a X^2 + b X + c I) in FP64, "
                                       "float64 D"}
    # the timed runs end with the one-layer model: recompute D with the full model for the error
    _, trD, trD2, info = api.expand_density(Hd, mu, kT, mref, prec=args.prec, out=D, ws=ws,
                                            want_info=True)
    Dg = D.double().cpu().numpy()

    if not args.no_gpu_baselines:
        th = torch.from_numpy(m.theta).to(dev)
        I = torch.eye(n, dtype=torch.float64, device=dev)

        def fp64_recursion():
            # plain FP64 recursion with vendor DGEMM (torch.matmul), same coefficients and rescale
            X = (info["scale"] * Hd + info["shift"] * I)
            A = torch.zeros_like(X)
            for a, b, cc, d in m.theta:
                A += d * X
                X = a * (X @ X) + b * X + cc * I
            return I - (A + X) if info["flipped"] else A + X

        ms64 = timed(fp64_recursion, 3, 1, torch)

        def eig_density():
            w, V = torch.linalg.eigh(Hd)
            f = torch.sigmoid(-(w - mu) / kT)
            return (V * f) @ V.T

        ms_eig = timed(eig_density, 2, 1, torch)
        # context for the MFMA fraction: the vendor FP16 GEMM (hipBLASLt via torch.matmul) on a
        # plain N x N x N product with random operands, same box and session
        ga = torch.randn(n, n, device=dev, dtype=torch.float16)
        gb = torch.randn(n, n, device=dev, dtype=torch.float16).t().contiguous()
        ms_gemm = timed(lambda: ga @ gb, 20, 3, torch)
        del ga, gb
        out["gpu_baselines"] = {
            "fp64_recursion_torch_dgemm_ms": ms64,
            "fp64_eigh_plus_assembly_ms": ms_eig,
            "vendor_fp16_gemm_tflops": 2.0 * n ** 3 / (ms_gemm * 1e-3) / 1e12,
            "speedup_vs_fp64_recursion": ms64 / ms,
            "speedup_vs_fp64_eigh": ms_eig / ms,
        }

    if not args.no_cpu_baseline:
        from oracle import fermi as F
        try:
            from threadpoolctl import threadpool_info
            threads = max(int(i.get("num_threads", 1)) for i in threadpool_info()
                          if i.get("user_api") == "blas")
        except Exception:
            threads = os.cpu_count()
        try:
            blas = sorted({i.get("internal_api", "?") for i in threadpool_info()
                           if i.get("user_api") == "blas"})
        except Exception:
            blas = []
        dts = []
        for _ in range(3):
            t0 = time.perf_counter()
            ref = F.density(H, mu, kT)
            dts.append(time.perf_counter() - t0)
        dt = sorted(dts)[1]
        out["cpu_baseline"] = {"value": 1.0 / dt, "unit": "density matrices/s", "cores": threads,
                               "nproc": os.cpu_count(), "blas": blas, "kind": "oracle",
                               "sample": "one full N=4096 matrix of the workload: LAPACK dsyevd "
                                         "eigendecomposition + V f V^T assembly in FP64 (numpy); "
                                         "median of 3 runs"}
        err = Dg - ref["D"]
        S_gpu = float(api.expand_entropy(Hd, mu, kT, mentref, ment.alpha, prec=args.prec,
                                         ws=ws)[0])
        S_fermi = float(api.expand_entropy(Hd, mu, kT, mref, 0.842704, prec=args.prec, ws=ws)[0])
        out["error_vs_oracle"] = {"fro_over_N": float(np.linalg.norm(err) / n),
                                  "max_abs": float(np.max(np.abs(err))),
                                  "norm2": norm2_sym(err, torch, dev),
                                  "abs_dTrD": abs(float(trD) - ref["trD"]),
                                  "abs_dTrD2": abs(float(trD2) - ref["trD2"]),
                                  "abs_dS": abs(S_gpu - ref["S"]), "S": ref["S"],
                                  "entropy_model": ment.name,
                                  "abs_dS_theta_fermi_reused": abs(S_fermi - ref["S"])}
        if Daff is not None:
            out["affine_form"]["fro_over_N_vs_oracle"] = float(np.linalg.norm(Daff - ref["D"]) / n)
        ec = Dcorr - ref["D"]
        out["final_correction"]["error_vs_oracle"] = {
            "fro_over_N": float(np.linalg.norm(ec) / n), "max_abs": float(np.max(np.abs(ec))),
            "norm2": norm2_sym(ec, torch, dev)}
    print(json.dumps(out), flush=True)


def launch_form(api, plan, want):
    """The launch form to time: the plan tuner's choice ("auto"), else the one asked for (the
    queue launch falls back to the per-layer launches where the device does not allow it).
    Returns (form, tuner's choice)."""
    tuned = plan.launch_form
    if want == "auto" or want == tuned:
        return tuned, tuned
    try:
        plan.set_launch(want)
        return want, tuned
    except api.FeError as e:
        print(f"batch launch form {want}: {e}", file=sys.stderr, flush=True)
        return tuned, tuned


def bench_batch(args, torch, api, models, workloads, dev):
    """1024 Hamiltonians, N_b ~ U{64..768}, one captured plan (a hipGraph: bounds, rescale, every
    layer of every matrix in one queue launch, or one grouped launch per layer, traces; its layer
    tile, 128 x 128 or 64 x 64, and its launch form chosen by the plan's autotuner, the other form
    timed beside it), the 40-layer (beta0 = 1e4, mu0 = 1/3) model, FP16x2 by default (BF16x2 misses the
    1e-5 bar on this batch: beta' reaches ~3700; --prec bf16x3, the three-part BF16 split, meets
    it). Sampled items are checked against the CPU oracle (eigendecomposition) in the
    cpu_baseline leg."""
    import numpy as np
    m = models.load("mlsp2_L40_b1e4_mu1third")
    t0 = time.perf_counter()
    items = workloads.batch_items(1024, 2000)
    print(f"batch inputs generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    mats = [dict(H=torch.from_numpy(it["H"]).to(dev), mu=it["mu"], kT=it["kT"]) for it in items]
    prec = args.prec
    plan = api.BatchPlan(mats, m, prec=prec)
    tile, tile_ms = plan.autotune()
    form, tuned_form = launch_form(api, plan, args.batch_launch)
    other = "queue" if form == "layers" else "layers"
    ms_other = None
    try:   # the other form, timed for comparison (the queue launch may be unavailable)
        plan.set_launch(other)
        ms_other = timed(plan.launch, args.steps, args.warmup, torch)
    except api.FeError as e:
        print(f"batch launch form {other}: {e}", file=sys.stderr, flush=True)
    plan.set_launch(form)
    ms = timed(plan.launch, args.steps, args.warmup, torch)
    status = plan.status.cpu().numpy()
    ns = np.array([it["n"] for it in items], dtype=np.float64)
    flop = float(np.sum(m.L * 2.0 * ns ** 3))
    out = {"metric": "density matrices/s (batch of 1024, N_b ~ U{64..768})",
           "value": 1024 / (ms * 1e-3), "unit": "density matrices/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "dtype": "bf16" if prec.startswith("bf16") else "f16",
           "data": "synthetic",
           "config": {"workload": "batch1024_banded_xi8_N64-768_seed2000", "items": 1024,
                      "layers": m.L, "coefficients": "mlsp2_L40_b1e4_mu1third",
                      "precision": prec},
           "tflops_algorithmic": flop / (ms * 1e-3) / 1e12,
           "status_nonzero": int(np.count_nonzero(status)),
           "tile_autotune": {"tile": tile, "ms_per_step": {str(k): v for k, v in tile_ms.items()}},
           "launch": {"form": form, "tuned": tuned_form,
                      "ms_per_step": {form: ms, other: ms_other}}}
    # the same batch over the model bank: each matrix runs the fewest layers valid for it
    bank_names = BANK
    bank = [models.load(x) for x in bank_names]
    plan.close()
    bplan = api.BatchPlan(mats, bank, prec=prec, ws=plan.ws)
    tile_b, tile_ms_b = bplan.autotune()
    form_b, tuned_b = launch_form(api, bplan, args.batch_launch)
    other_b = "queue" if form_b == "layers" else "layers"
    ms_b_other = None
    try:
        bplan.set_launch(other_b)
        ms_b_other = timed(bplan.launch, args.steps, args.warmup, torch)
    except api.FeError as e:
        print(f"batch launch form {other_b}: {e}", file=sys.stderr, flush=True)
    bplan.set_launch(form_b)
    ms_b = timed(bplan.launch, args.steps, args.warmup, torch)
    Ls = np.array([bank[k].L for k in bplan.chosen], dtype=np.float64)
    out["model_bank"] = {
        "value": 1024 / (ms_b * 1e-3), "unit": "density matrices/s", "ms_per_step": ms_b,
        "models": bank_names,
        "items_per_model": [int(np.sum(bplan.chosen == k)) for k in range(len(bank))],
        "tflops_algorithmic": float(np.sum(Ls * 2.0 * ns ** 3)) / (ms_b * 1e-3) / 1e12,
        "status_nonzero": int(np.count_nonzero(bplan.status.cpu().numpy())),
        "tile_autotune": {"tile": tile_b, "ms_per_step": {str(k): v for k, v in tile_ms_b.items()}},
        "launch": {"form": form_b, "tuned": tuned_b,
                   "ms_per_step": {form_b: ms_b, other_b: ms_b_other}}}
    if not args.no_cpu_baseline:
        from oracle import fermi as F
        order = np.argsort(ns)
        sample = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
        errs = []
        t0 = time.perf_counter()
        for b in sample:
            it = items[b]
            ref = F.density(it["H"], it["mu"], it["kT"])
            Dg = plan.D[b].double().cpu().numpy()
            Db = bplan.D[b].double().cpu().numpy()
            errs.append({"item": b, "N": it["n"],
                         "fro_over_N": float(np.linalg.norm(Dg - ref["D"]) / it["n"]),
                         "norm2": float(np.max(np.abs(np.linalg.eigvalsh(Dg - ref["D"])))),
                         "abs_dTrD": abs(float(plan.tr[b, 0]) - ref["trD"]),
                         "bank_model": bank_names[int(bplan.chosen[b])],
                         "bank_fro_over_N": float(np.linalg.norm(Db - ref["D"]) / it["n"])})
        dt = time.perf_counter() - t0
        out["error_vs_oracle_sampled"] = errs
        out["cpu_baseline"] = {"value": len(sample) / dt, "unit": "density matrices/s",
                               "kind": "oracle", "sample": "the smallest, median and largest "
                               "item of the batch (eigendecomposition + assembly, FP64)"}
    print(json.dumps(out), flush=True)


def bench_large(args, torch, api, models, workloads, dev):
    """One N = 16384 solve (h_ij = g_ij exp(-|i-j|/32), on-site U[-1,1], kT = 0.02, mu at 40%
    filling), the 40-layer (1e4, 1/3) model: density (FP16x2) and entropy (FP16x2, the trained
    40-layer entropy model; theta_fermi reused at alpha = 0.842704 beside it). mu is the oracle's
    40%-filling value from its stored reference for this input (tests/golden), against which the
    result is checked (sampled rows, probe products, traces, S), as well as against the FP64
    expansion on the GPU. Also timed with the model the bank selects (`model_bank`)."""
    import numpy as np
    m = models.load("mlsp2_L40_b1e4_mu1third")
    t0 = time.perf_counter()
    c = workloads.config_large_banded()
    n = c["H"].shape[0]
    Hd = torch.from_numpy(c["H"]).to(dev)
    del c["H"]
    # the oracle's reference for this seeded input (stored by tests/golden/make_large16384.py, which
    # calls only the oracle): its 40%-filling mu, eigenvalues, Tr D, sum D^2, S, sampled rows of D
    # and D v for probe vectors
    ref = np.load(LARGE_ORACLE) if os.path.exists(LARGE_ORACLE) else None
    kT = c["kT"]
    if ref is not None:
        mu = float(ref["mu"])
    else:
        lam = torch.linalg.eigvalsh(Hd).cpu().numpy()
        k = int(0.4 * n)
        mu = float(0.5 * (lam[k - 1] + lam[k]))
    print(f"large input generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    ws = api.Workspace(n)
    D = torch.empty((n, n), dtype=torch.float32, device=dev)
    mref = api.make_model(m.theta, m.beta0, m.mu0)
    tuned = api.autotune_input(Hd, mu, kT, mref, prec=args.prec, ws=ws)
    _, trD, trD2, info = api.expand_density(Hd, mu, kT, mref, prec=args.prec, out=D, ws=ws,
                                            want_info=True)
    steps = max(1, min(args.steps, 5))
    ms = timed(lambda: api.expand_density(Hd, mu, kT, mref, prec=args.prec, out=D, ws=ws),
               steps, 1, torch)
    ment = models.load("entropy_L40_b1e4_mu1third")
    mentref = api.make_model(ment.theta, ment.beta0, ment.mu0)
    ms_s = timed(lambda: api.expand_entropy(Hd, mu, kT, mentref, ment.alpha, prec=args.prec, ws=ws),
                 steps, 1, torch)
    S_ent = float(api.expand_entropy(Hd, mu, kT, mentref, ment.alpha, prec=args.prec, ws=ws)[0])
    S = float(api.expand_entropy(Hd, mu, kT, mref, 0.842704, prec=args.prec, ws=ws)[0])
    oracle_err = None
    if ref is not None:
        pfx = "mlsp2_L40_b1e4_mu1third"
        dv = (D.double() @ torch.from_numpy(ref["V"]).to(dev)).cpu().numpy()
        rows = D[torch.from_numpy(ref["rows"]).to(dev)].double().cpu().numpy()
        oracle_err = {
            "rows_max_abs_vs_exact": float(np.max(np.abs(rows - ref["exact_rows"]))),
            "probes_rel_vs_exact": float(np.linalg.norm(dv - ref["exact_probes"])
                                         / np.linalg.norm(ref["exact_probes"])),
            "abs_dTrD_vs_exact": abs(float(trD) - float(ref["exact_trD"])),
            "abs_dTrD_vs_recursion": abs(float(trD) - float(ref[f"{pfx}_trD"])),
            "abs_dS_theta_entropy_vs_exact": abs(S_ent - float(ref["exact_S"])),
            "abs_dS_theta_entropy_vs_recursion": abs(S_ent - float(ref["entropy_L40_b1e4_mu1third_S"]))
            if "entropy_L40_b1e4_mu1third_S" in ref.files else None,
            "abs_dS_theta_fermi_reused_vs_exact": abs(S - float(ref["exact_S"])),
            "S_exact": float(ref["exact_S"]),
            "sample": "the oracle's stored reference (tests/golden/large16384_oracle.npz): "
                      "8 rows of D, D v for 4 probe vectors, Tr D, S"}
    D64, trD64, _, _ = api.expand_density(Hd, mu, kT, mref, prec="fp64", ws=ws,
                                          out_dtype=torch.float64, want_info=True)
    S64 = float(api.expand_entropy(Hd, mu, kT, mref, 0.842704, prec="fp64", ws=ws)[0])
    torch.cuda.synchronize()
    err = (D.double() - D64)
    # the same solve with the model the bank selects for this matrix (selection inside the step)
    bank = [models.load(x) for x in BANK]
    bank_refs = [api.make_model(x.theta, x.beta0, x.mu0) for x in bank]
    kb = api.select_model(Hd, mu, kT, bank_refs, ws=ws)

    def bank_step():
        k = api.select_model(Hd, mu, kT, bank_refs, ws=ws)
        api.expand_density(Hd, mu, kT, bank_refs[k], prec=args.prec, out=D, ws=ws)
    ms_b = timed(bank_step, steps, 1, torch)
    Db64 = api.expand_density(Hd, mu, kT, bank_refs[kb], prec="fp64", ws=ws,
                              out_dtype=torch.float64)[0]
    torch.cuda.synchronize()
    bank_err = float(torch.linalg.norm(D.double() - Db64).item() / n)
    del Db64
    flop = m.L * 2.0 * n ** 3
    out = {"metric": "density matrices/s (single N = 16384 solve)",
           "value": 1000.0 / ms, "unit": "density matrices/s", "n_gpus": 1, "steps": steps,
           "warmup": 1, "ms_per_step": ms, "higher_is_better": True,
           "dtype": "f16" if args.prec == "fp16x2" else "bf16", "data": "synthetic",
           "config": {"workload": "banded_xi32_N16384_seed4_kT0.02_fill0.4", "N": n,
                      "layers": m.L, "coefficients": "mlsp2_L40_b1e4_mu1third",
                      "precision": args.prec, "mu": mu, "beta_p": info["beta_p"],
                      "schedule": api.autotune_lookup(n, args.prec, ws)},
           "autotune": tuned,
           "tflops_algorithmic": flop / (ms * 1e-3) / 1e12,
           "entropy_ms": ms_s, "entropy_model": ment.name,
           "trD": float(trD), "trD_target": 0.4 * n,
           "error_vs_oracle": oracle_err,
           "vs_fp64_expansion": {"fro_over_N": float(torch.linalg.norm(err).item() / n),
                                 "max_abs": float(err.abs().max().item()),
                                 "norm2": norm2_sym(err, torch, dev),
                                 "abs_dTrD": abs(float(trD) - float(trD64)),
                                 "abs_dS": abs(S - S64), "S": S},
           "model_bank": {"model": BANK[kb], "layers": bank[kb].L, "ms_per_step": ms_b,
                          "value": 1000.0 / ms_b,
                          "what": "model selection (bounds pass + read-back) + density expansion",
                          "fro_over_N_vs_fp64_expansion": bank_err}}
    print(json.dumps(out), flush=True)


def bench_filling(args, torch, api, models, workloads, dev):
    """The N = 4096 Anderson workload at half filling (Tr D = 2048) instead of a given mu: the
    chemical potential by safeguarded Newton iterations (Sec. IV.3) from the midpoint of the
    Gershgorin interval, each iterate one full expansion. Checked against the oracle's mu
    (bisection on the eigenvalues) and density in the cpu_baseline leg."""
    import numpy as np
    m = models.load("mlsp2_L26_b1500_mu1third")
    c = workloads.config_anderson_4096()
    H = c["H"]
    n = H.shape[0]
    n_occ = 0.5 * n
    Hd = torch.from_numpy(H).to(dev)
    ws = api.Workspace(n)
    D = torch.empty((n, n), dtype=torch.float32, device=dev)
    mref = api.make_model(m.theta, m.beta0, m.mu0)
    res = {}

    def solve():
        res["r"] = api.expand_density_filling(Hd, n_occ, c["kT"], mref, prec=args.prec, out=D,
                                              ws=ws)
    ms = timed(solve, max(1, min(args.steps, 10)), 1, torch)
    _, mu, iters, tr, tr2, info = res["r"]
    out = {"metric": "density matrices/s at a prescribed occupation (Newton mu)",
           "value": 1000.0 / ms, "unit": "density matrices/s", "n_gpus": 1,
           "steps": max(1, min(args.steps, 10)), "warmup": 1, "ms_per_step": ms,
           "higher_is_better": True, "dtype": "f16" if args.prec == "fp16x2" else "bf16",
           "data": "synthetic",
           "config": {"workload": "anderson_cubic_16x16x16_periodic_N4096_t-1_W1_kT0.05_half_filling",
                      "N": n, "n_occ": n_occ, "layers": m.L,
                      "coefficients": "mlsp2_L26_b1500_mu1third", "precision": args.prec},
           "newton_iterations": iters, "mu": mu, "abs_trD_minus_n_occ": abs(float(tr) - n_occ)}
    # the same solve with the bank model selected at the Newton start (the Gershgorin midpoint)
    _, rinfo = api.rescale(Hd, 0.0, c["kT"], mref, want_X0=False, ws=ws)
    mu_start = 0.5 * (rinfo["emin"] + rinfo["emax"])
    bank = [models.load(x) for x in BANK]
    bank_refs = [api.make_model(x.theta, x.beta0, x.mu0) for x in bank]
    Db = torch.empty_like(D)

    def solve_bank():
        k = api.select_model(Hd, mu_start, c["kT"], bank_refs, ws=ws)
        res["b"] = (k, api.expand_density_filling(Hd, n_occ, c["kT"], bank_refs[k], prec=args.prec,
                                                  out=Db, ws=ws))
    ms_b = timed(solve_bank, max(1, min(args.steps, 10)), 1, torch)
    kb, (_, mu_b, iters_b, tr_b, _, _) = res["b"]
    out["model_bank"] = {"model": BANK[kb], "layers": bank[kb].L, "ms_per_step": ms_b,
                         "value": 1000.0 / ms_b, "newton_iterations": iters_b, "mu": mu_b,
                         "abs_trD_minus_n_occ": abs(float(tr_b) - n_occ),
                         "what": "model selection at the Newton start + Newton solve"}
    if not args.no_cpu_baseline:
        from oracle import fermi as F
        t0 = time.perf_counter()
        lam = np.linalg.eigvalsh(H)
        mu_ref = F.mu_for_filling(lam, n_occ, c["kT"])
        ref = F.density(H, mu_ref, c["kT"])
        dt = time.perf_counter() - t0
        err = D.double().cpu().numpy() - ref["D"]
        out["error_vs_oracle"] = {"fro_over_N": float(np.linalg.norm(err) / n),
                                  "norm2": norm2_sym(err, torch, dev),
                                  "abs_dmu": abs(mu - mu_ref)}
        err_b = Db.double().cpu().numpy() - ref["D"]
        out["model_bank"]["error_vs_oracle"] = {"fro_over_N": float(np.linalg.norm(err_b) / n),
                                                "abs_dmu": abs(mu_b - mu_ref)}
        out["cpu_baseline"] = {"value": 1.0 / dt, "unit": "density matrices/s", "kind": "oracle",
                               "sample": "the full matrix: eigenvalues, bisection for mu, then "
                                         "eigendecomposition + assembly at that mu (FP64)"}
    print(json.dumps(out), flush=True)


def bench_train(args, torch, api, models, workloads, dev):
    """Coefficient training at the 40-layer, beta0 = 1e4, mu0 = 1/3 setting (Sec. III.C): the
    scalar Levenberg-Marquardt fit to the Fermi target on 8192 points (FP64 Jacobian kernel) from
    the SP2 start, timed to its stop; then forward + backward passes of the FP32 matrix recursion
    (torch.autograd.Function over fe_matrix_forward / fe_matrix_backward) over 64 matrices of the
    random dense family at N = 256 (seeds 3000 + m, kT = 0.1, half filling), loss = sum of squared
    errors against GPU FP64 eigendecomposition densities."""
    import numpy as np

    from paper_2605_08523_amd import training
    L, beta0, mu0 = 40, 1e4, 1.0 / 3.0
    torch.cuda.synchronize()
    # iterations until the sample points' max error is below 1e-7 (the paper: "a few hundred"
    # with geodesic acceleration, Sec. III.C)
    t0 = time.perf_counter()
    _, rep7, ok7 = training.train_coeffs(L, beta0, mu0, n_points=8192, max_iter=10000, tol=1e-7)
    dt7 = time.perf_counter() - t0
    t0 = time.perf_counter()
    th, rep, ok = training.train_coeffs(L, beta0, mu0, n_points=8192, max_iter=10000, tol=1e-10)
    dt = time.perf_counter() - t0
    out = {"metric": "LM iterations/s of the 40-layer coefficient fit (8192 points)",
           "value": rep["iters"] / dt, "unit": "LM iterations/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "train_L40_b1e4_mu1third_8192pts", "layers": L, "beta0": beta0,
                      "mu0": mu0, "points": 8192},
           "iterations": rep["iters"], "seconds_to_stop": dt,
           "ms_per_iteration": 1e3 * dt / max(1, rep["iters"]), "converged": bool(ok),
           "max_error_grid": rep["max_err_grid"],
           "to_1e-7": {"iterations": rep7["iters"], "seconds": dt7, "reached": bool(ok7),
                       "max_error_grid": rep7["max_err_grid"]}}
    # matrix-level passes
    n, nm, kT = 256, 64, 0.1
    model = api.make_model(th, beta0, mu0)
    X0s, refs = [], []
    for k in range(nm):
        H = torch.from_numpy(workloads.random_dense(n, 3000 + k)).to(dev)
        lam, V = torch.linalg.eigh(H)
        mu = float(0.5 * (lam[n // 2 - 1] + lam[n // 2]))
        X0, info = api.rescale(H, mu, kT, model, want_X0=True)
        D = (V * torch.sigmoid(-(lam - mu) / kT)) @ V.T
        refs.append(torch.eye(n, device=dev, dtype=torch.float64) - D if info["flipped"] else D)
        X0s.append(X0.contiguous())
    theta = torch.tensor(th, dtype=torch.float64, requires_grad=True)

    def fwd_bwd():
        theta.grad = None
        loss = 0.0
        for X0, Dr in zip(X0s, refs):
            P = training.matrix_recursion(theta, X0)
            loss = loss + ((P.double() - Dr) ** 2).sum()
        loss.backward()
        return float(loss.detach())
    loss0 = fwd_bwd()
    steps = max(2, min(args.steps, 10))
    ms_mb = timed(fwd_bwd, steps, 1, torch)
    out["matrix_fwd_bwd"] = {"matrices": nm, "N": n, "layers": L, "ms_per_pass": ms_mb,
                             "ms_per_matrix": ms_mb / nm, "loss": loss0,
                             "rms_error": float(np.sqrt(loss0 / (nm * n * n))),
                             "grad_norm": float(theta.grad.norm())}
    # the fit refined on the 64 matrices (fe_train_coeffs with the matrix set: combined objective,
    # matrix term through the FP32 forward / backward kernels), from the fitted coefficients
    mats = [(X0, Dr.contiguous()) for X0, Dr in zip(X0s, refs)]
    t0 = time.perf_counter()
    thm, repm, _ = training.train_coeffs(L, beta0, mu0, n_points=8192, max_iter=1, tol=1e-10,
                                         theta_init=th, mats=mats, mat_iters=10, mat_weight=1.0)
    dtm = time.perf_counter() - t0
    out["matrix_set_refinement"] = {
        "matrices": nm, "N": n, "iterations": repm["mat_iters"], "kept": repm["mat_accepted"],
        "seconds": dtm, "matrix_loss_start": repm["mat_loss_start"],
        "matrix_loss_end": repm["mat_loss_end"],
        "grid_max_error_before": rep["max_err_grid"],
        "grid_max_error_after": repm["max_err_grid"],
        "what": "loss = sum_m ||P(X0_m) - Dref_m||_F^2, P by the FP32 kernels; Dref from FP64 "
                "eigendecompositions on the GPU; weight 1 against the 8192 points' squares"}
    print(json.dumps(out), flush=True)


def bench_variants(args, torch, api, models, workloads, dev):
    """Skip-SP2 (k = K = 1) and Max-SP2 on the N = 4096 Anderson workload (Sec. III.A), each the
    App. C embedding of the 22-layer beta0 = 600, mu0 = 1/3 model (the same function as that MLSP2
    model): per layer one square-only split MFMA pass and one HBM-bound combine pass.
    Timed beside the fused MLSP2 path on the same matrix; errors against the oracle's exact D."""
    import numpy as np

    from paper_2605_08523_amd import variants
    base = models.load("mlsp2_L22_b600_mu1third")
    c = workloads.config_anderson_4096()
    H = c["H"]
    n = H.shape[0]
    Hd = torch.from_numpy(H).to(dev)
    mu, kT = c["mu"], c["kT"]
    ws = api.Workspace(n)
    D = torch.empty((n, n), dtype=torch.float32, device=dev)
    mref = api.make_model(base.theta, base.beta0, base.mu0)
    fams = {"max": variants.embed_mlsp2(base, "max"), "skip": variants.embed_mlsp2(base, "skip")}
    scratch = {k: torch.empty(variants.scratch_bytes(n, q), dtype=torch.uint8, device=dev)
               for k, q in fams.items()}
    if args.profile:
        for _ in range(args.warmup + args.steps):
            for k, q in fams.items():
                variants.expand_density_variant(Hd, mu, kT, q, prec=args.prec, out=D,
                                                scratch=scratch[k], ws=ws)
        torch.cuda.synchronize()
        print("profile run done", flush=True)
        return
    ms_m = timed(lambda: api.expand_density(Hd, mu, kT, mref, prec=args.prec, out=D, ws=ws),
                 args.steps, args.warmup, torch)
    res = {}
    ref = None
    if not args.no_cpu_baseline:
        from oracle import fermi as F
        ref = F.density(H, mu, kT)
    np_ = -(-n // 128) * 128
    upper = np_ * (np_ + 64) // 2            # elements of the upper 64 x 64 tiles
    for k, q in fams.items():
        ms = timed(lambda: variants.expand_density_variant(Hd, mu, kT, q, prec=args.prec, out=D,
                                                           scratch=scratch[k], ws=ws),
                   args.steps, args.warmup, torch)
        L = q.L
        # combine passes, per upper element: each stored state it reads once (4 B), each
        # accumulator it writes (4 B), hi/lo of the tile and its mirror (8 B); the result pass
        # reads the output terms and writes D for both triangles (8 B)
        if k == "max":
            per_layer = [4 * (i + 1) + 8 for i in range(L)]
            final = 4 * (L + 1) + 8
        else:
            per_layer = [4 * (1 + (1 if i > 0 else 0)) + 4 + 8 for i in range(L)]
            final = 4 * 2 + 8
        comb_bytes = upper * (sum(per_layer) + final)
        r = {"ms_per_step": ms, "value": 1000.0 / ms, "layers": L, "coefficients": len(q.coef),
             "combine_algorithmic_bytes_per_step": comb_bytes,
             "slowdown_vs_fused_mlsp2": ms / ms_m}
        if ref is not None:
            r["error_vs_oracle_fro_over_N"] = float(np.linalg.norm(D.double().cpu().numpy() -
                                                                   ref["D"]) / n)
        res[k] = r
    # per-layer time of the Skip-SP2 path (square + combine; constant per layer) by the same
    # difference as the headline: (t(L layers) - t(1 layer)) / (L - 1), HIP events on the stream
    q1 = variants.embed_mlsp2(api.make_model(base.theta[-1:], base.beta0, base.mu0), "skip")
    ms1 = timed(lambda: variants.expand_density_variant(Hd, mu, kT, q1, prec=args.prec, out=D,
                                                        scratch=scratch["skip"], ws=ws),
                args.steps, args.warmup, torch)
    L = fams["skip"].L
    layer_ms = (res["skip"]["ms_per_step"] - ms1) / (L - 1)
    achieved = 2.0 * n ** 3 / (layer_ms * 1e-3) / 1e12
    out = {"metric": "density matrices/s, Skip-SP2 / Max-SP2 embeddings of the selected model",
           "value": res["skip"]["value"], "unit": "density matrices/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["skip"]["ms_per_step"],
           "higher_is_better": True, "dtype": "f16" if args.prec == "fp16x2" else "bf16",
           "data": "synthetic",
           "config": {"workload": "anderson_cubic_16x16x16_periodic_N4096_t-1_W1_kT0.05_mu0",
                      "N": n, "model": "App. C embedding of mlsp2_L22_b600_mu1third",
                      "precision": args.prec},
           "skip_sp2_k1_K1": res["skip"], "max_sp2": res["max"], "fused_mlsp2_ms": ms_m,
           "roofline": {"kernel": "Skip-SP2 layer: k_square (split MFMA square, K-split last "
                                  "round) + k_combine", "bound": "mfma", "achieved": achieved,
                        "peak": PEAK_TFLOPS[args.prec], "unit": "TFLOP/s",
                        "frac": achieved / PEAK_TFLOPS[args.prec], "traffic": None,
                        "layer_ms": layer_ms,
                        "method": f"HIP events: (t(L={L}) - t(L=1)) / {L - 1}, algorithmic 2 N^3"}}
    print(json.dumps(out), flush=True)


def bench_small(args, torch, api, models, workloads, dev):
    """The small FP64 configuration: N = 128 dense random (seed 0), kT = 0.1, mu for half filling
    (Tr D = 64, found by the library's Newton iteration in FP64), the 30-layer beta0 = 1500,
    mu0 = 1/3 model, FP64 products in one workgroup's LDS (`k_small_f64`). One solve per step
    (launch-latency bound: one CU of 256 works); density and entropy timed."""
    import numpy as np
    m = models.load("mlsp2_L30_b1500_mu1third")
    c = workloads.config_small_dense(0)
    H, kT = c["H"], c["kT"]
    n = H.shape[0]
    Hd = torch.from_numpy(H).to(dev)
    mref = api.make_model(m.theta, m.beta0, m.mu0)
    ws = api.Workspace(n)
    D = torch.empty((n, n), dtype=torch.float64, device=dev)
    _, mu, iters, _, _, _ = api.expand_density_filling(Hd, c["n_target"], kT, mref, prec="fp64",
                                                       out_dtype=torch.float64, ws=ws)
    _, trD, trD2, info = api.expand_density(Hd, mu, kT, mref, prec="fp64", out=D, ws=ws,
                                            want_info=True)
    steps = max(args.steps, 200)
    ms = timed(lambda: api.expand_density(Hd, mu, kT, mref, prec="fp64", out=D, ws=ws), steps,
               max(args.warmup, 10), torch)
    ms_s = timed(lambda: api.expand_entropy(Hd, mu, kT, mref, 0.842704, prec="fp64", ws=ws), steps,
                 max(args.warmup, 10), torch)
    flop = m.L * 2.0 * n ** 3
    out = {"metric": "density matrices/s (one N = 128 FP64 solve)", "value": 1000.0 / ms,
           "unit": "density matrices/s", "n_gpus": 1, "steps": steps, "warmup": max(args.warmup, 10),
           "ms_per_step": ms, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "random_dense_N128_seed0_kT0.1_half_filling", "N": n,
                      "layers": m.L, "coefficients": m.name, "mu": mu, "newton_iterations": iters,
                      "beta_p": info["beta_p"]},
           "tflops_algorithmic": flop / (ms * 1e-3) / 1e12,
           "roofline": {"kernel": "k_small_f64 (whole recursion in one workgroup's LDS)",
                        "bound": "latency", "achieved": flop / (ms * 1e-3) / 1e12,
                        "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                        "frac": flop / (ms * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"],
                        "note": "one workgroup on one of the 256 CUs; the step is the launch "
                                "sequence of bounds, rescale, recursion and reduction"},
           "entropy_ms": ms_s, "trD": float(trD)}
    D_g = D.cpu().numpy()
    if not args.no_cpu_baseline:
        from oracle import fermi as F
        lam = np.linalg.eigvalsh(H)
        mu_ref = F.mu_for_filling(lam, c["n_target"], kT)
        dts = []
        for _ in range(20):
            t0 = time.perf_counter()
            ref = F.density(H, mu_ref, kT)
            dts.append(time.perf_counter() - t0)
        dt = sorted(dts)[len(dts) // 2]
        err = D_g - F.density(H, mu, kT)["D"]
        out["cpu_baseline"] = {"value": 1.0 / dt, "unit": "density matrices/s", "kind": "oracle",
                               "cores": os.cpu_count(),
                               "sample": "the full N = 128 matrix: eigendecomposition + assembly "
                                         "(FP64, numpy), median of 20 runs"}
        out["error_vs_oracle"] = {"fro_over_N": float(np.linalg.norm(err) / n),
                                  "max_abs": float(np.max(np.abs(err))),
                                  "abs_dTrD": abs(float(trD) - ref["trD"]),
                                  "abs_dmu": abs(mu - mu_ref)}
    print(json.dumps(out), flush=True)


def bench_sweep(args, torch, api, models, workloads, dev):
    """The paper's timing experiment (Sec. V.D): wall clock of a 26-layer evaluation with the
    printed (beta0 = 1500, mu0 = 1/3) model on random dense symmetric matrices of growing N,
    against diagonalization-based density matrices (FP64 and FP32 eigh + V f V^T) on the same
    GPU. kT is set per matrix so that beta' = 600 (inside the model's validity, beta' <= 1000),
    mu at the middle of the Gershgorin interval. Errors against the FP64 diagonalization."""
    import numpy as np
    m = models.load("mlsp2_L26_b1500_mu1third")
    mref = api.make_model(m.theta, m.beta0, m.mu0)
    rows = []
    for n in (256, 512, 1024, 2048, 4096, 8192):
        H = workloads.random_dense(n, 50 + n)
        r = np.abs(H).sum(axis=1) - np.abs(np.diag(H))
        lo, hi = float(np.min(np.diag(H) - r)), float(np.max(np.diag(H) + r))
        mu, kT = 0.5 * (lo + hi), (hi - lo) / 600.0
        Hd = torch.from_numpy(H).to(dev)
        ws = api.Workspace(n)
        D = torch.empty((n, n), dtype=torch.float32, device=dev)
        steps = max(2, min(args.steps, 10))
        ms = timed(lambda: api.expand_density(Hd, mu, kT, mref, prec=args.prec, out=D, ws=ws),
                   steps, 1, torch)

        def eig(dtype):
            Hc = Hd.to(dtype)
            w, V = torch.linalg.eigh(Hc)
            f = torch.sigmoid(-(w - mu) / kT)
            return (V * f) @ V.T
        reps = 2 if n >= 4096 else 3
        ms64 = timed(lambda: eig(torch.float64), reps, 1, torch)
        ms32 = timed(lambda: eig(torch.float32), reps, 1, torch)
        D64 = eig(torch.float64)
        D32 = eig(torch.float32)
        torch.cuda.synchronize()
        rows.append({"N": n, "ms": ms, "schedule": api.autotune_lookup(n, args.prec, ws),
                     "tflops_algorithmic": m.L * 2.0 * n ** 3 / (ms * 1e-3) / 1e12,
                     "eigh_fp64_ms": ms64, "eigh_fp32_ms": ms32,
                     "speedup_vs_eigh_fp64": ms64 / ms, "speedup_vs_eigh_fp32": ms32 / ms,
                     "fro_over_N_vs_eigh_fp64": float(torch.linalg.norm(D.double() - D64).item() / n),
                     "fro_over_N_eigh_fp32_vs_fp64": float(torch.linalg.norm(D32.double() - D64).item() / n)})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        ws.close()
        del Hd, D, D64, D32
        torch.cuda.empty_cache()
    out = {"metric": "ms per density matrix vs N (26 layers) and speedup over eigh",
           "value": rows[-2]["speedup_vs_eigh_fp64"], "unit": "x vs FP64 eigh at N = 4096",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f16" if args.prec == "fp16x2" else "bf16",
           "data": "synthetic",
           "config": {"workload": "random_dense_sweep_N256-8192_beta600", "layers": m.L,
                      "coefficients": m.name, "precision": args.prec},
           "rows": rows}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
