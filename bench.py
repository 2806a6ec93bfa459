"""Throughput benchmark of the fused stream-collide sweep on one MI355X.

Headline workload: D3Q19 TRT (Lambda = 3/16, tau_e = 0.8) on a 256^3 channel
(solid planes y = 0 and y = 255, periodic x and z), constant body force 1e-6
along x, rho = 1 with seeded uniform +-1e-3 velocity noise, PDFs in FP64.
A step is one fused stream-pull-collide launch over the whole lattice (the
inputs are resident in HBM).  The JSON line also carries the FP32-storage
run of the same workload, the Q-stream copy reference, the D3Q27 cumulant
(FP32/BF16/FP16 storage, 384^3), the D3Q19 SRT forward+adjoint gradient
(128^3, FP32, tape every 20 steps) and the D3Q27 MRT (512^3, FP16 vs FP64).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]
                       [--no-cpu-baseline] [--only fp32,aa,copy,methods,c1,c3,c4,c5]
       python bench.py trace-summary DIR      (rocprofv3 --kernel-trace output,
                                                per kernel and grid size)
       python bench.py pmc-summary FETCH_DIR WRITE_DIR [--write]
                                              (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
                                               runs; --write updates profiles/)
"""

import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12          # MI355X HBM3E, bytes/s
METRIC = "MLUPS & % HBM roofline: D3Q19/D3Q27 fwd+adjoint, FP64 vs FP32/FP16-store"
BYTES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    """Hash of the kernel sources and the build flags (build.py)."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2001_11806_amd")
    for f in sorted(glob.glob(os.path.join(pkg, "csrc", "*"))) + [os.path.join(pkg, "build.py")]:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(name):
    """Per-launch HBM bytes from a committed rocprofv3 counter summary, or
    None when it is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


class Timer:
    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def __enter__(self):
        self.a = self.torch.cuda.Event(enable_timing=True)
        self.b = self.torch.cuda.Event(enable_timing=True)
        self.torch.cuda.synchronize()
        self.a.record(self.stream)
        return self

    def __exit__(self, *exc):
        self.b.record(self.stream)
        self.torch.cuda.synchronize()
        self.ms = self.a.elapsed_time(self.b)


def run_forward(torch, LBM, inputs, stencil, method, dtype, dims, rates, mask, u, F=None, profile=None,
                steps=100, warmup=10, pattern=0, cs_smag=0.0):
    lbm = LBM(stencil, method, dtype, dims, rates["omega"], rates.get("omega_bulk", 1.0),
              rates.get("omega_odd", 0.0), rates.get("magic", 0.0), rates.get("omega_hi", (1.0,) * 4),
              mask=mask, pattern=pattern, cs_smag=cs_smag)
    if F is not None:
        lbm.set_force(F)
    if profile is not None:
        lbm.set_force(profile=profile)
    lbm.init_equilibrium(None, torch.from_numpy(u))
    lbm.step(warmup)
    with Timer(torch, lbm.stream) as t:
        lbm.step(steps)
    cells = dims[0] * dims[1] * dims[2]
    fluid = cells - (int(mask.sum()) if mask is not None else 0)
    Q = {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27}[stencil]
    per_launch = fluid * 2 * Q * BYTES[dtype] + (cells if mask is not None else 0)
    sec = t.ms / 1e3
    res = {
        "mlups": cells * steps / sec / 1e6,
        "fluid_mlups": fluid * steps / sec / 1e6,
        "ms_per_step": t.ms / steps,
        "algorithmic_bytes_per_launch": per_launch,
        "achieved_GBps": per_launch * steps / sec / 1e9,
    }
    res["hbm_frac"] = res["achieved_GBps"] * 1e9 / PEAK_HBM
    cons = lbm.conserved()
    res["mass"] = float(cons[0])
    rr, uu = lbm.macroscopic(dtype=torch.float64)
    res["u_out"], res["rho_out"] = uu, rr
    lbm.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--short", action="store_true",
                    help="profiling runs: C3 and C5 for 20 steps instead of their configured 500 and 1000 "
                         "(their error figures then refer to 20 steps)")
    ap.add_argument("--only", default="", help="comma list of extras to run (fp32,aa,copy,methods,c1,c3,c4,c5)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the multi-GPU halo exchange is not built "
              "(design only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2001_11806_amd import inputs
    from paper_2001_11806_amd.lbm import LBM, copy_q, stream_aa_q, stream_q

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_start = time.time()

    # ------------------------------------------------------------ headline
    n = 256
    trt = dict(omega=1 / 0.8, magic=3 / 16, omega_odd=0.0)
    mask, _, u = inputs.channel_flow(n, seed=2, amp=1e-3)
    F = np.array([1e-6, 0.0, 0.0])
    log("C2 D3Q19 TRT 256^3 f64: %d warmup + %d timed steps" % (args.warmup, args.steps))
    head = run_forward(torch, LBM, inputs, "D3Q19", "TRT", "f64", (n, n, n), trt, mask, u, F=F,
                       steps=args.steps, warmup=args.warmup)
    u64 = head.pop("u_out")
    head.pop("rho_out")
    log("  %.0f MLUPS, %.0f GB/s" % (head["mlups"], head["achieved_GBps"]))
    extras = {}
    only = set(filter(None, args.only.split(",")))
    want = (lambda k: not args.no_extras and (not only or k in only))

    if want("fp32"):
        log("C2 D3Q19 TRT 256^3 f32-shifted")
        r32 = run_forward(torch, LBM, inputs, "D3Q19", "TRT", "f32", (n, n, n), trt, mask, u, F=F,
                          steps=args.steps, warmup=args.warmup)
        u32 = r32.pop("u_out")
        r32.pop("rho_out")
        fl = torch.from_numpy(mask == 0).to(dev)
        d = (u32.double() - u64.double())[:, fl]
        r32["rel_l2_u_vs_f64_same_gpu"] = float(d.norm() / u64.double()[:, fl].norm())
        extras["c2_d3q19_trt_256_f32"] = r32
        log("  %.0f MLUPS, rel err u %.2e" % (r32["mlups"], r32["rel_l2_u_vs_f64_same_gpu"]))
    if want("aa"):
        log("C2 D3Q19 TRT 256^3 f64, AA pattern (one array)")
        raa = run_forward(torch, LBM, inputs, "D3Q19", "TRT", "f64", (n, n, n), trt, mask, u, F=F,
                          steps=args.steps, warmup=args.warmup, pattern=1)
        uaa = raa.pop("u_out")
        raa.pop("rho_out")
        raa["u_equal_to_two_array_run"] = bool(torch.equal(uaa, u64))
        extras["c2_d3q19_trt_256_f64_aa"] = raa
        log("  %.0f MLUPS, %.0f GB/s, identical to two-array: %s" % (raa["mlups"], raa["achieved_GBps"],
                                                                    raa["u_equal_to_two_array_run"]))
    del u64
    torch.cuda.empty_cache()

    if want("copy"):
        extras.update(bench_copies(torch, copy_q, stream_q, stream_aa_q, Timer, dev))

    if want("c3"):
        # the full 500-step run in every storage type; FP64 on the same GPU
        # (parity-checked against the oracle) is the reference for the errors
        n3 = 384
        T3 = 20 if args.short else 500
        log("C3 D3Q27 cumulant 384^3, %d steps: building solenoidal field" % T3)
        modes = inputs.solenoidal_modes(seed=3)
        u3 = inputs.solenoidal_velocity(n3, modes, dtype=np.float32)
        cum = dict(omega=1 / 0.55, omega_bulk=1.0, omega_hi=(1.0,) * 4)
        ref = None
        for dt in ("f64", "f32", "bf16", "f16"):
            r = run_forward(torch, LBM, inputs, "D3Q27", "CUMULANT", dt, (n3, n3, n3), cum, None, u3,
                            steps=T3 - 5, warmup=5)
            uo, ro = r.pop("u_out"), r.pop("rho_out")
            if ref is None:
                ref = (uo, ro)
            else:
                r["rel_l2_u_vs_f64_%d_steps" % T3] = float((uo - ref[0]).norm() / ref[0].norm())
                r["rel_l2_rho_minus_1_vs_f64_%d_steps" % T3] = float((ro - ref[1]).norm() / (ref[1] - 1).norm())
                # what the figures mean: FP32 against its 1e-5 bar; whether the
                # storage resolves the density deviation at all (error < 10 %)
                if dt == "f32":
                    r["u_within_fp32_bar_1e-5"] = r["rel_l2_u_vs_f64_%d_steps" % T3] <= 1e-5
                r["rho_minus_1_resolved"] = r["rel_l2_rho_minus_1_vs_f64_%d_steps" % T3] < 0.1
            extras["c3_d3q27_cumulant_384_%s" % dt] = r
            log("  %s: %.0f MLUPS, %.0f GB/s%s" % (dt, r["mlups"], r["achieved_GBps"], "" if dt == "f64" else
                ", rel L2 vs FP64: u %.2e, rho-1 %.2e" % (r["rel_l2_u_vs_f64_%d_steps" % T3],
                                                          r["rel_l2_rho_minus_1_vs_f64_%d_steps" % T3])))
            del uo, ro
            torch.cuda.empty_cache()
        del ref, u3
        torch.cuda.empty_cache()

    if want("methods"):
        extras["method_comparison"] = bench_methods(torch, LBM, inputs, Timer, run_forward)

    if want("c1"):
        extras["c1_d2q9_srt_64_f64"] = bench_c1(torch, LBM, inputs, Timer)

    if want("c4"):
        extras["c4_d3q19_srt_adjoint_128_f32"] = bench_adjoint(torch, LBM, inputs, Timer)
        aa = bench_adjoint(torch, LBM, inputs, Timer, pattern=1)
        aa["gradients_equal_to_two_array"] = aa["dL_dF"] == extras["c4_d3q19_srt_adjoint_128_f32"]["dL_dF"]
        extras["c4_d3q19_srt_adjoint_128_f32_aa"] = aa
        torch.cuda.empty_cache()

    if want("c5"):
        n5 = 512
        T5 = 20 if args.short else 1000
        log("C5 D3Q27 MRT 512^3, %d steps: building noise field" % T5)
        u5 = inputs.uniform_noise_velocity((n5, n5, n5), 1e-3, 5, None, dtype=np.float32)
        prof = inputs.kolmogorov_force_profile(n5, 1e-6)
        mrt = dict(omega=1 / 0.55, omega_bulk=1.2, omega_hi=(1.0,) * 4)
        ref = None
        for dt in ("f64", "f16"):
            r = run_forward(torch, LBM, inputs, "D3Q27", "MRT", dt, (n5, n5, n5), mrt, None, u5, profile=prof,
                            steps=T5 - 5, warmup=5)
            uo, ro = r.pop("u_out"), r.pop("rho_out")
            if ref is None:
                ref = uo
            else:
                r["rel_l2_u_vs_f64_same_gpu_%d_steps" % T5] = float((uo - ref).norm() / ref.norm())
            extras["c5_d3q27_mrt_512_%s" % dt] = r
            log("  %s: %.0f MLUPS, %.0f GB/s%s" % (dt, r["mlups"], r["achieved_GBps"], "" if dt == "f64" else
                ", rel L2 u vs FP64 after %d steps %.2e" % (T5, r["rel_l2_u_vs_f64_same_gpu_%d_steps" % T5])))
            del uo, ro
            torch.cuda.empty_cache()
        del ref, u5

    # ------------------------------------------------------------ CPU oracle
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(inputs)

    # the headline, fluid cells only, and its copy line / counter figures
    extras["c2_d3q19_trt_256_f64"] = {"fluid_mlups": head["fluid_mlups"], "achieved_GBps": head["achieved_GBps"],
                                      "algorithmic_bytes_per_launch": head["algorithmic_bytes_per_launch"]}
    attach_lines(extras)
    line, sline, prof = MATCH["c2_d3q19_trt_256_f64"]
    traffic = read_traffic(prof)
    result = {
        "metric": METRIC,
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded channel flow (numpy PCG64), no dataset",
        "config": {"workload": "D3Q19 TRT (magic 3/16, tau 0.8) 256^3 channel, bounce-back walls y=0,255, "
                               "force 1e-6 x, FP64 PDFs, two-array pull",
                   "lattice": [n, n, n], "stencil": "D3Q19", "method": "TRT", "storage": "f64",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": head["achieved_GBps"], "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                     "frac": head["hbm_frac"], "traffic": traffic,
                     "algorithmic_bytes_per_launch": head["algorithmic_bytes_per_launch"],
                     "kernel": "k_sweep<D3Q19, TRT, double>",
                     # attainable line: the 19-plane FP64 copy of the same size in the
                     # sweep's launch shape, same run; and a plain device-to-device memcpy
                     "copy_line_GBps": extras.get(line, {}).get("GBps"),
                     "frac_of_copy_line": (head["achieved_GBps"] / extras[line]["GBps"]
                                           if line in extras else None),
                     # the same sweep's access pattern without its arithmetic
                     "stream_line_GBps": extras.get(sline, {}).get("GBps"),
                     "frac_of_stream_line": (head["achieved_GBps"] / extras[sline]["GBps"]
                                             if sline in extras else None),
                     "memcpy_d2d_GBps": extras.get("memcpy_d2d_4GiB", {}).get("GBps")},
        "cpu_baseline": cpu,
        "extras": extras,
        "wall_s": round(time.time() - t_start, 1),
    }
    print(json.dumps(result))


# Bandwidth references, each in the launch shape of the sweep compared with
# it (resident wavefronts per CU: the LDS-capped count the sweep runs with,
# or the count its registers allow when that is lower; threads per block =
# the sweep's row segment) and with its store type (non-temporal above
# 512 MiB), over arrays of the workload's size and element type:
#   copy_*   Q read and Q write SoA streams, element i to element i (the
#            paper's multi-stream copy benchmark, Sec. V-A, Tab. III);
#   stream_* the sweep's pull access pattern without its arithmetic:
#            periodic pull streaming dst[q][x] = src[q][x - c_q];
#   aa_*     the AA pattern's data movement without arithmetic: its even and
#            odd in-place kernels alternating on one array.
# Key -> (kind, stencil, lattice edge, storage, element bytes, waves per CU
# (0 = full occupancy), threads per block).
LINES = {
    # C2 FP64 two-array sweep (12 waves per CU)
    "copy_q19_f64_256_w12_b256": ("copy", "D3Q19", 256, "f64", 8, 12, 256),
    "stream_d3q19_f64_256_w12_b256": ("stream", "D3Q19", 256, "f64", 8, 12, 256),
    # C2 FP64 AA sweeps (full occupancy = 16 waves per CU at their 120-128 VGPRs)
    "copy_q19_f64_256_w16_b256": ("copy", "D3Q19", 256, "f64", 8, 16, 256),
    "stream_d3q19_f64_256_w16_b256": ("stream", "D3Q19", 256, "f64", 8, 16, 256),
    "aa_d3q19_f64_256_w16_b256": ("aa", "D3Q19", 256, "f64", 8, 16, 256),
    # C2 FP32 two-array sweep (16 waves per CU)
    "copy_q19_f32_256_w16_b256": ("copy", "D3Q19", 256, "f32", 4, 16, 256),
    "stream_d3q19_f32_256_w16_b256": ("stream", "D3Q19", 256, "f32", 4, 16, 256),
    # C3 FP64 cumulant, the error reference (12 waves per CU)
    "copy_q27_f64_384_w12_b384": ("copy", "D3Q27", 384, "f64", 8, 12, 384),
    "stream_d3q27_f64_384_w12_b384": ("stream", "D3Q27", 384, "f64", 8, 12, 384),
    # C3 FP32 cumulant (full occupancy: five 384-cell blocks per CU)
    "copy_q27_f32_384_w0_b384": ("copy", "D3Q27", 384, "f32", 4, 0, 384),
    "stream_d3q27_f32_384_w0_b384": ("stream", "D3Q27", 384, "f32", 4, 0, 384),
    # C3 BF16 / FP16 cumulant (128-cell segments, full occupancy)
    "copy_q27_f16_384_w0_b128": ("copy", "D3Q27", 384, "f16", 2, 0, 128),
    "stream_d3q27_f16_384_w0_b128": ("stream", "D3Q27", 384, "f16", 2, 0, 128),
    # C5 FP64 MRT (256-cell segments, 12 waves per CU: the register limit)
    "copy_q27_f64_512_w12_b256": ("copy", "D3Q27", 512, "f64", 8, 12, 256),
    "stream_d3q27_f64_512_w12_b256": ("stream", "D3Q27", 512, "f64", 8, 12, 256),
    # C5 FP16 MRT (512-cell rows, full occupancy)
    "copy_q27_f16_512_w0_b512": ("copy", "D3Q27", 512, "f16", 2, 0, 512),
    "stream_d3q27_f16_512_w0_b512": ("stream", "D3Q27", 512, "f16", 2, 0, 512),
}
# workload -> (matching copy line, matching pull-stream line, committed
# counter summary of its sweep kernel)
MATCH = {
    "c2_d3q19_trt_256_f64": ("copy_q19_f64_256_w12_b256", "stream_d3q19_f64_256_w12_b256",
                             "sweep_d3q19_trt_256_f64_traffic.txt"),
    "c2_d3q19_trt_256_f32": ("copy_q19_f32_256_w16_b256", "stream_d3q19_f32_256_w16_b256",
                             "sweep_d3q19_trt_256_f32_traffic.txt"),
    "c2_d3q19_trt_256_f64_aa": ("copy_q19_f64_256_w16_b256", "stream_d3q19_f64_256_w16_b256",
                                "sweep_aa_d3q19_trt_256_f64_traffic.txt"),
    "c3_d3q27_cumulant_384_f64": ("copy_q27_f64_384_w12_b384", "stream_d3q27_f64_384_w12_b384",
                                  "sweep_d3q27_cumulant_384_f64_traffic.txt"),
    "c3_d3q27_cumulant_384_f32": ("copy_q27_f32_384_w0_b384", "stream_d3q27_f32_384_w0_b384",
                                  "sweep_d3q27_cumulant_384_f32_traffic.txt"),
    "c3_d3q27_cumulant_384_bf16": ("copy_q27_f16_384_w0_b128", "stream_d3q27_f16_384_w0_b128",
                                   "sweep_d3q27_cumulant_384_bf16_traffic.txt"),
    "c3_d3q27_cumulant_384_f16": ("copy_q27_f16_384_w0_b128", "stream_d3q27_f16_384_w0_b128",
                                  "sweep_d3q27_cumulant_384_f16_traffic.txt"),
    "c5_d3q27_mrt_512_f64": ("copy_q27_f64_512_w12_b256", "stream_d3q27_f64_512_w12_b256",
                             "sweep_d3q27_mrt_512_f64_traffic.txt"),
    "c5_d3q27_mrt_512_f16": ("copy_q27_f16_512_w0_b512", "stream_d3q27_f16_512_w0_b512",
                             "sweep_d3q27_mrt_512_f16_traffic.txt"),
    "c4_d3q19_srt_adjoint_128_f32": (None, None, "adj_sweep_aa_d3q19_srt_128_f32_traffic.txt"),
}
# the AA workload's own access-pattern line
AA_LINE = {"c2_d3q19_trt_256_f64_aa": "aa_d3q19_f64_256_w16_b256"}


def bench_copies(torch, copy_q, stream_q, stream_aa_q, Timer, dev):
    """Copy and pull-stream lines of every configured workload, plus two
    copies that owe nothing to this library: hipMemcpyAsync device to device
    (called directly in the HIP runtime torch loaded) and torch's
    Tensor.copy_, each on a 4 GiB buffer."""
    import ctypes
    out = {}
    st = torch.cuda.current_stream(dev)
    for key, (kind, stencil, n, dt, eb, waves, block) in LINES.items():
        q = 19 if stencil == "D3Q19" else 27
        N = n ** 3
        src = torch.empty(q * N * eb // 4, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src) if kind != "aa" else None

        def run(i):
            if kind == "copy":
                copy_q(src, dst, N, q, eb, st, waves, block)
            elif kind == "stream":
                stream_q(src, dst, (n, n, n), stencil, eb, st, waves, block)
            else:   # even and odd kernels alternating, in place
                stream_aa_q(src, (n, n, n), stencil, eb, i & 1, st, waves, block)
        for i in range(4):
            run(i)
        with Timer(torch, st) as t:
            for i in range(20):
                run(i)
        gbps = 2 * q * N * eb * 20 / (t.ms / 1e3) / 1e9
        out[key] = {"GBps": gbps, "hbm_frac": gbps * 1e9 / PEAK_HBM}
        log("%s: %.0f GB/s" % (key, gbps))
        del src, dst
        torch.cuda.empty_cache()
    nbytes = 4 << 30
    src = torch.empty(nbytes // 4, dtype=torch.int32, device=dev).fill_(1)
    dst = torch.empty_like(src)
    try:
        hip = ctypes.CDLL("libamdhip64.so.7", mode=os.RTLD_NOLOAD)   # the runtime already in the process
        hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                       ctypes.c_void_p]
        hip.hipMemcpyAsync.restype = ctypes.c_int

        def memcpy():
            rc = hip.hipMemcpyAsync(dst.data_ptr(), src.data_ptr(), nbytes, 3, st.cuda_stream)  # 3: D2D
            if rc != 0:
                raise RuntimeError("hipMemcpyAsync returned %d" % rc)
        for _ in range(2):
            memcpy()
        with Timer(torch, st) as t:
            for _ in range(10):
                memcpy()
        gbps = 2 * nbytes * 10 / (t.ms / 1e3) / 1e9
        out["memcpy_d2d_4GiB"] = {"GBps": gbps, "hbm_frac": gbps * 1e9 / PEAK_HBM}
        log("hipMemcpyAsync D2D 4 GiB: %.0f GB/s" % gbps)
    except (OSError, RuntimeError) as e:
        out["memcpy_d2d_4GiB"] = {"GBps": None, "error": str(e)}
    for _ in range(2):
        dst.copy_(src)
    with Timer(torch, st) as t:
        for _ in range(10):
            dst.copy_(src)
    gbps = 2 * nbytes * 10 / (t.ms / 1e3) / 1e9
    out["torch_copy_4GiB"] = {"GBps": gbps, "hbm_frac": gbps * 1e9 / PEAK_HBM}
    log("torch copy_ 4 GiB: %.0f GB/s" % gbps)
    del src, dst
    torch.cuda.empty_cache()
    return out


def attach_lines(extras):
    """Per workload: the matching copy and pull-stream lines, the fraction of
    each reached, and the counter-measured HBM bytes per launch while the
    committed summary matches the kernel sources."""
    for w, (line, sline, prof) in MATCH.items():
        if w not in extras:
            continue
        r = extras[w]
        aline = AA_LINE.get(w)
        if aline and aline in extras and "achieved_GBps" in r:
            r["aa_line"] = aline
            r["frac_of_aa_line"] = r["achieved_GBps"] / extras[aline]["GBps"]
        if line and line in extras and "achieved_GBps" in r:
            r["copy_line"] = line
            r["frac_of_copy_line"] = r["achieved_GBps"] / extras[line]["GBps"]
        if sline and sline in extras and "achieved_GBps" in r:
            r["stream_line"] = sline
            r["frac_of_stream_line"] = r["achieved_GBps"] / extras[sline]["GBps"]
        tr = read_traffic(prof)
        r["traffic"] = tr
        if tr is not None and "algorithmic_bytes_per_launch" in r:
            r["traffic_over_algorithmic"] = tr / r["algorithmic_bytes_per_launch"]


def bench_methods(torch, LBM, inputs, Timer, run_forward):
    """Per-method throughput on the same lattice (the paper compares TRT,
    Smagorinsky, weighted MRT, cumulant and entropic KBC kernels with the AA
    pattern and finds them memory bound): D3Q19 256^3 channel FP64 with AA,
    and D3Q27 256^3 periodic FP32 two-array."""
    out = {}
    n = 256
    mask, _, u = inputs.channel_flow(n, seed=2, amp=1e-3)
    F = np.array([1e-6, 0.0, 0.0])
    base = dict(omega=1 / 0.8, omega_bulk=1.2, magic=3 / 16, omega_odd=0.0, omega_hi=(1.0,) * 4)
    for name, method, extra in (("SRT", "SRT", {}), ("TRT", "TRT", {}), ("MRT", "MRT", {}),
                                ("SRT_Smagorinsky", "SRT", {"cs_smag": 0.1}),
                                ("MRT_Smagorinsky", "MRT", {"cs_smag": 0.1}), ("KBC", "KBC", {})):
        r = run_forward(torch, LBM, inputs, "D3Q19", method, "f64", (n, n, n), dict(base, **extra), mask, u, F=F,
                        steps=50, warmup=5, pattern=1, cs_smag=extra.get("cs_smag", 0.0))
        r.pop("u_out")
        out["D3Q19_f64_AA_" + name] = {"mlups": r["mlups"], "GBps": r["achieved_GBps"]}
        log("  D3Q19 f64 AA %-16s %7.0f MLUPS %6.0f GB/s" % (name, r["mlups"], r["achieved_GBps"]))
    u27 = inputs.uniform_noise_velocity((n, n, n), 1e-3, 6, None, dtype=np.float32)
    for name, method, rates in (("SRT", "SRT", base), ("TRT", "TRT", base), ("MRT", "MRT", base),
                                ("CUMULANT", "CUMULANT", dict(base, omega_bulk=1.0)),
                                ("CUMULANT_general_rates", "CUMULANT", dict(base, omega_bulk=1.0,
                                                                            omega_hi=(1.2, 1.1, 1.0, 1.3))),
                                ("KBC", "KBC", base)):
        r = run_forward(torch, LBM, inputs, "D3Q27", method, "f32", (n, n, n), rates, None, u27, steps=50, warmup=5)
        r.pop("u_out")
        out["D3Q27_f32_" + name] = {"mlups": r["mlups"], "GBps": r["achieved_GBps"]}
        log("  D3Q27 f32    %-22s %7.0f MLUPS %6.0f GB/s" % (name, r["mlups"], r["achieved_GBps"]))
    torch.cuda.empty_cache()
    return out


def bench_c1(torch, LBM, inputs, Timer):
    """C1: D2Q9 SRT 64^2 Taylor-Green, FP64, 1000 steps; launch-latency bound,
    so the graph replay (launch_mode 0) is timed beside direct launches."""
    rho, u = inputs.taylor_green_2d(64, 0.01)
    out = {}
    for mode, name in ((0, "graph"), (1, "direct")):
        lbm = LBM("D2Q9", "SRT", "f64", (64, 64, 1), 1 / 0.8, launch_mode=mode)
        lbm.init_equilibrium(torch.from_numpy(rho), torch.from_numpy(u))
        lbm.step(64)
        with Timer(torch, lbm.stream) as t:
            lbm.step(1000)
        lbm.close()
        out[name + "_mlups"] = 64 * 64 * 1000 / (t.ms / 1e3) / 1e6
        out[name + "_us_per_step"] = t.ms
    log("C1 D2Q9 64^2: graph %.0f MLUPS (%.2f us/step), direct %.0f MLUPS (%.2f us/step)" % (
        out["graph_mlups"], out["graph_us_per_step"], out["direct_mlups"], out["direct_us_per_step"]))
    return out


def bench_adjoint(torch, LBM, inputs, Timer, pattern=0):
    """C4: D3Q19 SRT 128^3 channel with 5% spheres, FP32, 200 steps forward,
    tape every 20, adjoint back to t=0 (segment recompute included); pattern 1
    runs the forward sweep and the adjoint in one array each (AA)."""
    n, T, k = 128, 200, 20
    log("C4 D3Q19 SRT adjoint 128^3 f32, T=%d, k=%d, %s" % (T, k, "AA" if pattern else "two arrays"))
    mask = inputs.sphere_channel_mask(n, seed=4)
    u0 = inputs.uniform_noise_velocity((n, n, n), 1e-3, 4, mask, dtype=np.float32)
    lbm = LBM("D3Q19", "SRT", "f32", (n, n, n), 1 / 0.8, mask=mask, checkpoint_every=k, max_tape_steps=T,
              pattern=pattern)
    lbm.set_force([1e-5, 0, 0])
    u0t = torch.from_numpy(u0).cuda()
    fl = torch.from_numpy(mask == 0).cuda()
    for rep in range(2):       # first pass warms up
        lbm.init_equilibrium(None, u0t)
        with Timer(torch, lbm.stream) as tf:
            lbm.step(T)
        _, uT = lbm.macroscopic(dtype=torch.float32)
        g = torch.zeros_like(uT)
        g[0, :, :, -1] = 2 * uT[0, :, :, -1] * fl[:, :, -1]
        with Timer(torch, lbm.stream) as tb:
            lbm.adjoint_seed(g)
            lbm.adjoint_step(T)
            du, _, dF = lbm.adjoint_grads(dtype=torch.float32)
    lbm.close()
    cells = n ** 3
    fluid = cells - int(mask.sum())
    per_step = fluid * (2 * 19 * 4) * 2 + fluid * 3 * 19 * 4 + 3 * cells   # fwd + recompute + adjoint
    sec = (tf.ms + tb.ms) / 1e3
    log("  %.0f MLUPS effective (forward %.1f ms, backward %.1f ms)" % (cells * T / sec / 1e6, tf.ms, tb.ms))
    return {"fwd_adjoint_mlups": cells * T / sec / 1e6, "forward_ms": tf.ms, "backward_ms": tb.ms,
            "algorithmic_GBps": per_step * T / sec / 1e9, "dL_dF": [float(v) for v in dF],
            "dL_du0_norm": float(du.double().norm())}


def cpu_baseline(inputs):
    """The C++ FP64 oracle as it stands (plain loops, OpenMP over rows) on all
    the host threads it sees, on bounded samples: the headline workload on
    its full 256^3 channel for as many steps as fit in about 12 s (at least
    one, at most 100), then a 384 x 384 x 16 slab of the cumulant workload
    and a 512 x 512 x 16 slab of the Kolmogorov MRT workload, six steps each
    (their full lattices would need 24 GB and 58 GB of host memory for two
    FP64 arrays).  Every sample is timed after one untimed step that touches
    both arrays.  Returns the headline figure and the per-workload samples."""
    from oracle import cpu as ocpu, run as orun
    threads = ocpu.num_threads()
    host = {"threads": threads, "os_cpu_count": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}

    def timed(cfg, P, steps, mask=None, force=None):
        t0 = time.time()
        P = ocpu.run(cfg, P, steps, mask, force)
        return P, time.time() - t0

    n = 256
    mask, _, u = inputs.channel_flow(n, seed=2, amp=1e-3)
    cfg = orun.Config("D3Q19", "TRT", dict(omega=1 / 0.8, magic=3 / 16, omega_odd=0.0))
    F = np.array([1e-6, 0.0, 0.0])
    P = ocpu.init_equilibrium(cfg, None, u, mask)
    del u
    # each call allocates its output array, so a call's time is a fixed
    # first-touch cost plus the steps: estimate the per-step time from the
    # difference of a one-step and a three-step call
    P, t1 = timed(cfg, P, 1, mask, F)
    P, t3 = timed(cfg, P, 3, mask, F)
    steps = int(max(1, min(100, 12.0 // max((t3 - t1) / 2, 1e-3))))
    P, dt = timed(cfg, P, steps, mask, F)
    del P
    head = n ** 3 * steps / dt / 1e6
    log("CPU oracle, C2 256^3: %.1f MLUPS (%d steps, %.1f s, %d threads)" % (head, steps, dt, threads))
    samples = {"c2_d3q19_trt_256_f64": {"mlups": head, "steps": steps, "seconds": dt, "lattice": [n, n, n]}}
    cells = np.arange(384 * 384 * 16)
    u3 = inputs.solenoidal_velocity_at(384, inputs.solenoidal_modes(seed=3), cells).reshape(3, 16, 384, 384)
    c3 = orun.Config("D3Q27", "CUMULANT", dict(omega=1 / 0.55, omega_bulk=1.0, omega_hi=(1.0,) * 4))
    P, _ = timed(c3, ocpu.init_equilibrium(c3, None, u3), 1)
    P, dt = timed(c3, P, 6)
    samples["c3_d3q27_cumulant_f64"] = {"mlups": u3[0].size * 6 / dt / 1e6, "steps": 6, "seconds": dt,
                                        "lattice": [384, 384, 16]}
    del P, u3
    u5 = inputs.uniform_noise_velocity((512, 512, 16), 1e-3, 5, None)
    c5 = orun.Config("D3Q27", "MRT", dict(omega=1 / 0.55, omega_bulk=1.2, omega_hi=(1.0,) * 4))
    prof = inputs.kolmogorov_force_profile(512, 1e-6)
    P, _ = timed(c5, ocpu.init_equilibrium(c5, None, u5), 1, None, prof)
    P, dt = timed(c5, P, 6, None, prof)
    samples["c5_d3q27_mrt_f64"] = {"mlups": u5[0].size * 6 / dt / 1e6, "steps": 6, "seconds": dt,
                                   "lattice": [512, 512, 16]}
    del P, u5
    log("CPU oracle samples: C3 %.2f MLUPS, C5 %.2f MLUPS" % (samples["c3_d3q27_cumulant_f64"]["mlups"],
                                                              samples["c5_d3q27_mrt_f64"]["mlups"]))
    return {"value": head, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "C++ FP64 oracle (OpenMP, %d threads), the headline D3Q19 TRT channel on its full 256^3 "
                      "lattice, %d steps in %.1f s" % (threads, steps, samples["c2_d3q19_trt_256_f64"]["seconds"]),
            "host": host, "samples": samples}


# ---------------------------------------------------------------- profile summaries
# Counter summaries the benchmark reads back (MATCH): file -> (kernel symbol
# as rocprofv3 names it, dispatch grid size in threads, algorithmic bytes per
# launch, description).  C2: fluid = 256^3 - 2 * 256^2 cells plus one flag
# byte per cell; C3 / C5 are periodic (no flags).
_C2_FLUID = 256 ** 3 - 2 * 256 ** 2
PROFILED = {
    "sweep_d3q19_trt_256_f64_traffic.txt": (
        "k_sweep<D3Q19, TRT, double, NT>", 256 ** 3, 2 * 19 * 8 * _C2_FLUID + 256 ** 3,
        "k_sweep<D3Q19, TRT, double> on the 256^3 channel (C2 FP64, two arrays)"),
    "sweep_d3q19_trt_256_f32_traffic.txt": (
        "k_sweep<D3Q19, TRT, float, NT>", 256 ** 3, 2 * 19 * 4 * _C2_FLUID + 256 ** 3,
        "k_sweep<D3Q19, TRT, float> on the 256^3 channel (C2 FP32-shifted, two arrays)"),
    "sweep_aa_d3q19_trt_256_f64_traffic.txt": (
        "k_sweep_aa_*<D3Q19, TRT, double, NT>", 256 ** 3, 2 * 19 * 8 * _C2_FLUID + 256 ** 3,
        "k_sweep_aa_even / k_sweep_aa_odd<D3Q19, TRT, double> on the 256^3 channel (C2 FP64, AA), "
        "averaged over both kernels"),
    "sweep_d3q27_cumulant_384_f64_traffic.txt": (
        "k_sweep<D3Q27, CUMULANT, double, NT>", 384 ** 3, 2 * 27 * 8 * 384 ** 3,
        "k_sweep<D3Q27, CUMULANT, double> on the 384^3 periodic box (C3 FP64 reference)"),
    "sweep_d3q27_cumulant_384_f32_traffic.txt": (
        "k_sweep<D3Q27, CUMULANT, float, NT>", 384 ** 3, 2 * 27 * 4 * 384 ** 3,
        "k_sweep<D3Q27, CUMULANT, float> on the 384^3 periodic box (C3 FP32)"),
    "sweep_d3q27_cumulant_384_bf16_traffic.txt": (
        "k_sweep<D3Q27, CUMULANT, bf16, NT>", 384 ** 3, 2 * 27 * 2 * 384 ** 3,
        "k_sweep<D3Q27, CUMULANT, bf16> on the 384^3 periodic box (C3 BF16)"),
    "sweep_d3q27_cumulant_384_f16_traffic.txt": (
        "k_sweep<D3Q27, CUMULANT, f16, NT>", 384 ** 3, 2 * 27 * 2 * 384 ** 3,
        "k_sweep<D3Q27, CUMULANT, f16> on the 384^3 periodic box (C3 FP16)"),
    "sweep_d3q27_mrt_512_f64_traffic.txt": (
        "k_sweep<D3Q27, MRT, double, NT>", 512 ** 3, 2 * 27 * 8 * 512 ** 3,
        "k_sweep<D3Q27, MRT, double> on the 512^3 periodic box (C5 FP64)"),
    "sweep_d3q27_mrt_512_f16_traffic.txt": (
        "k_sweep<D3Q27, MRT_UNIT, f16, NT>", 512 ** 3, 2 * 27 * 2 * 512 ** 3,
        "k_sweep<D3Q27, MRT_UNIT, f16> (MRT with unit higher-order rates) on the 512^3 periodic box (C5 FP16)"),
    "adj_sweep_aa_d3q19_srt_128_f32_traffic.txt": (
        "k_adj_sweep_aa<D3Q19, float, *, 0>", 128 ** 3, (19 * 4 + 2 * 19 * 4 + 1) * 128 ** 3,
        "k_adj_sweep_aa<D3Q19, float> (even and odd) on the 128^3 channel with spheres (C4 adjoint step; "
        "algorithmic bytes taken as (Q s + 2 Q r + 1) N over all cells)"),
}


def _db_rows(directory, query):
    """Rows of `query` over every rocprofv3 result database (*_results.db,
    SQLite) below directory."""
    import sqlite3
    rows = []
    for path in sorted(glob.glob(os.path.join(directory, "**", "*_results.db"), recursive=True)):
        con = sqlite3.connect(path)
        try:
            rows.extend(con.execute(query).fetchall())
        finally:
            con.close()
    return rows


# method template codes of the sweeps (collide.h) and storage types
_METHOD_CODES = {"0": "SRT", "1": "TRT", "2": "MRT", "3": "CUMULANT", "4": "SRT_SMAG", "5": "MRT_SMAG",
                 "6": "CUMULANT_GEN", "7": "KBC", "8": "MRT_UNIT"}
_MANGLED_TYPES = {"d": "double", "f": "float", "DF16_": "f16", "DF16b": "bf16"}


def _kernel(name, mangled=""):
    """Kernel symbol without namespaces, argument list and template noise;
    sweep templates as k_sweep<stencil, method, storage[, NT]> (from the
    mangled symbol where the profiler's demangling of 16-bit types fails)."""
    import re
    m = re.match(r"_ZN3lbm\d+(k_sweep\w*)INS_\d(D\w+?)ELi(\d+)E(DF16_|DF16b|d|f)Li(\d)E", mangled or name)
    if m:     # symbols the profiler could not demangle (16-bit float types)
        return "%s<%s, %s, %s%s>" % (m.group(1), m.group(2), _METHOD_CODES.get(m.group(3), m.group(3)),
                                    _MANGLED_TYPES[m.group(4)], ", NT" if m.group(5) == "1" else "")
    name = re.sub(r"\(.*$", "", name.replace("lbm::", "").replace("(anonymous namespace)::", ""))
    name = re.sub(r"^void ", "", name)
    m = re.match(r"(k_sweep\w*)<(D\w+), (\d+), ([^,>]+), (\d)>$", name)
    if m:
        name = "%s<%s, %s, %s%s>" % (m.group(1), m.group(2), _METHOD_CODES.get(m.group(3), m.group(3)),
                                    m.group(4).replace("__bf16", "bf16").replace("_Float16", "f16"),
                                    ", NT" if m.group(5) == "1" else "")
    name = name.replace("unsigned long", "uint64").replace("unsigned int", "uint32").replace("unsigned short",
                                                                                              "uint16")
    return name


def trace_summary(directory):
    """Per (kernel, grid size) statistics of a rocprofv3 --kernel-trace run:
    calls, average / min / max duration in ns, workgroup size, VGPRs
    allocated per lane.  rocprofv3 derives its VGPR count from the code
    object's granule field in units of 4 registers, while gfx950 allocates
    VGPRs in granules of 8, so the allocation is twice the figure it records
    (k_sweep<D3Q19, TRT, double>: 74 VGPRs in the code object, 80
    allocated, 40 recorded)."""
    groups = {}
    q = ("select k.name, s.kernel_name, k.grid_x, k.workgroup_x, k.vgpr_count, k.duration from kernels k "
         "left join kernel_symbols s on k.kernel_id = s.kernel_id")
    for name, mangled, grid, wg, vgpr, dur in _db_rows(directory, q):
        g = groups.setdefault((_kernel(name, mangled or ""), int(grid)), {"d": [], "wg": wg, "vgpr": vgpr})
        g["d"].append(int(dur))
    lines = [" calls       avg_ns       min_ns       max_ns        grid    wg  vgpr  kernel"]
    for (k, grid), g in sorted(groups.items(), key=lambda kv: -sum(kv[1]["d"])):
        d = g["d"]
        vg = 2 * int(g["vgpr"]) if g["vgpr"] is not None else "-"
        lines.append("%6d %12.0f %12d %12d %11d %5s %5s  %s" % (len(d), sum(d) / len(d), min(d), max(d), grid,
                                                             g["wg"], vg, k))
    return "\n".join(lines)


def _counter_means(directory, counter):
    acc = {}
    q = ("select c.kernel_name, s.kernel_name, c.grid_size, c.value from counters_collection c "
         "left join kernel_symbols s on c.kernel_id = s.kernel_id where c.counter_name = '%s'" % counter)
    for name, mangled, grid, value in _db_rows(directory, q):
        acc.setdefault((_kernel(name, mangled or ""), int(grid)), []).append(float(value))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def _copy_bytes(kernel, grid):
    """Bytes one k_copy_q<E, Q> dispatch reads (and writes) over `grid` cells."""
    import re
    m = re.match(r"k_copy_q<uint(\d+), (\d+)(, \d)?>$", kernel)
    return None if not m else int(m.group(1)) // 8 * int(m.group(2)) * grid


def pmc_summary(fetch_dir, write_dir, write_files=False):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of two rocprofv3 --pmc runs,
    scaled by what the same counters read for the plain copy kernels of known
    size in the same runs; with write_files, the summaries of PROFILED."""
    fetch, write = _counter_means(fetch_dir, "FETCH_SIZE"), _counter_means(write_dir, "WRITE_SIZE")
    fs, ws = [], []
    for key in fetch:
        b = _copy_bytes(*key)
        if b and key in write:
            fs.append(b / 1024 / fetch[key])
            ws.append(b / 1024 / write[key])
    if not fs:
        raise SystemExit("no k_copy_q dispatch in the counter runs: nothing to calibrate with")
    f_scale, w_scale = sum(fs) / len(fs), sum(ws) / len(ws)
    out = ["# scale factors from %d copy kernels: fetch %.4f (spread %.4f..%.4f), write %.4f (%.4f..%.4f)"
           % (len(fs), f_scale, min(fs), max(fs), w_scale, min(ws), max(ws)),
           "  fetch_KiB     write_KiB       grid  kernel"]
    for key in sorted(fetch, key=lambda k: -(fetch[k] + write.get(k, 0))):
        out.append("%11.1f %13.1f %10d  %s" % (fetch[key], write.get(key, float("nan")), key[1], key[0]))
    if write_files:
        import fnmatch
        for fname, (kern, grid, alg, desc) in PROFILED.items():
            keys = [k for k in fetch if fnmatch.fnmatchcase(k[0], kern) and k[1] == grid and k in write]
            if not keys:
                out.append("# %s: kernel %s (grid %d) not in the runs" % (fname, kern, grid))
                continue
            fk = sum(fetch[k] for k in keys) / len(keys)
            wk = sum(write[k] for k in keys) / len(keys)
            hbm = (fk * f_scale + wk * w_scale) * 1024
            with open(os.path.join(ROOT, "profiles", fname), "w") as fh:
                fh.write("# HBM traffic of %s (one launch)\n" % desc)
                fh.write("# commands (MI355X machine, repository root R, TMPDIR=/tmp; one counter per run):\n"
                         "#   rocprofv3 --pmc FETCH_SIZE -d $R/gpurun_out/pmc_fetch -o fetch -- python $R/bench.py "
                         "--no-cpu-baseline --short --steps 5 --warmup 1 --only copy,fp32,aa,c3,c4,c5\n"
                         "#   rocprofv3 --pmc WRITE_SIZE -d $R/gpurun_out/pmc_write -o write -- python $R/bench.py "
                         "--no-cpu-baseline --short --steps 5 --warmup 1 --only copy,fp32,aa,c3,c4,c5\n"
                         "#   python bench.py pmc-summary gpurun_out/pmc_fetch gpurun_out/pmc_write --write\n"
                         "# counters are KiB per dispatch, averaged over the dispatches of the kernel at this\n"
                         "# grid size, scaled by what they read for the copy kernels k_copy_q of known size\n"
                         "# in the same runs\n")
                fh.write("# fetch scale %.4f, write scale %.4f; algorithmic bytes per launch %d\n"
                         % (f_scale, w_scale, alg))
                fh.write("# scaled HBM bytes / algorithmic bytes = %.4f\n" % (hbm / alg))
                fh.write("source_sha=%s\nfetch_kib_per_launch=%.1f\nwrite_kib_per_launch=%.1f\n"
                         "fetch_scale=%.6f\nwrite_scale=%.6f\nalgorithmic_bytes_per_launch=%d\n"
                         "hbm_bytes_per_launch=%.1f\n" % (source_hash(), fk, wk, f_scale, w_scale, alg, hbm))
            out.append("# wrote profiles/%s: %.4e bytes per launch, %.4f x algorithmic" % (fname, hbm, hbm / alg))
    return "\n".join(out)


def pmc_table(directory):
    """Average of every counter of a rocprofv3 --pmc run per (kernel, grid
    size), one row per kernel, and for the sweeps the per-cell figures of
    the SQ counters (instructions per lane = per cell, VALU busy share)."""
    acc = {}
    q = ("select c.kernel_name, s.kernel_name, c.grid_size, c.counter_name, c.value from counters_collection c "
         "left join kernel_symbols s on c.kernel_id = s.kernel_id")
    for name, mangled, grid, cname, value in _db_rows(directory, q):
        acc.setdefault((_kernel(name, mangled or ""), int(grid)), {}).setdefault(cname, []).append(float(value))
    lines = []
    for (k, grid), cs in sorted(acc.items(), key=lambda kv: -kv[0][1]):
        if "sweep" not in k and "copy_q" not in k and "stream_q" not in k and "adj" not in k:
            continue
        m = {c: sum(v) / len(v) for c, v in cs.items()}
        extra = ""
        if m.get("SQ_WAVES"):
            w = m["SQ_WAVES"]
            per = ["%s/wave %.0f" % (c[3:], m[c] / w) for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD",
                                                               "SQ_INSTS_VMEM_WR") if c in m]
            if "SQ_INSTS_VALU" in m and m.get("GRBM_GUI_ACTIVE"):
                # issue share of the VALU ceiling (one wave64 VALU instruction per CU
                # and clock); GRBM_GUI_ACTIVE is summed over the 8 XCDs
                per.append("VALU issue %.1f %% of the ceiling" % (100 * m["SQ_INSTS_VALU"] / 256
                                                                  / (m["GRBM_GUI_ACTIVE"] / 8)))
            extra = "  " + ", ".join(per)
        lines.append("%-44s grid %10d  %s%s" % (k, grid, " ".join("%s=%.4g" % kv for kv in sorted(m.items())), extra))
    return "\n".join(lines)


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "pmc-table":
        print(pmc_table(sys.argv[2]))
    elif len(sys.argv) > 2 and sys.argv[1] == "trace-summary":
        print(trace_summary(sys.argv[2]))
    elif len(sys.argv) > 3 and sys.argv[1] == "pmc-summary":
        print(pmc_summary(sys.argv[2], sys.argv[3], write_files="--write" in sys.argv[4:]))
    else:
        main()
