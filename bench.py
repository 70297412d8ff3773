#!/usr/bin/env python3
"""Benchmark of the randomized Chebyshev Fermi-operator hot path on one MI355X.

Headline workload (sc64): periodic simple-cubic tight binding, L = 64 (262,144
sites), t = -1, onsite disorder uniform in [-0.5, 0.5], kT = 0.02|t|, mu = 0.3,
2048 Chebyshev terms, 256 Rademacher probes, FP64.  One timed step is one
fermi_moments call: coefficients, 2047 fused Chebyshev steps with moments and
the density accumulator, moment reductions, traces and the density blocks.

metric: Chebyshev H.V step GB/s = algorithmic bytes of all H.V steps of the timed
calls / wall time of those calls.  Algorithmic bytes per step: H_hat values,
column indices and row pointers once, y_k once, y_{k-1} once, y_{k+1} once,
the packed probe bits once, and the accumulator read and written once per
update (one update per three steps, plus one at the last step).

Also reported on the same line:
  roofline      for the Chebyshev step kernel, from HIP events around its launches
  sc64_fp32     the same call with FP32 steps: time and differences against FP64
  cpu_baseline  the FP64 oracle's Chebyshev steps on the host (bounded sample)
A "step" of the line (steps, ms_per_step) is one fermi_moments call, i.e. one pass of
the whole hot path; each holds chebyshev_steps_per_step = 2047 Chebyshev steps, whose
mean kernel time is roofline.mean_launch_us.

  energy_force  energy + gradient + Hellmann-Feynman forces on the 16,000-atom
                Cu-like cluster (8000 terms, 256 probes), FP64, FP32, BF16 MFMA and BF16
                MFMA with H_hat split into hi + lo BF16 parts (bf16x2), with the doubled
                moments (the library default), and FP64 with the direct
                recurrence, with the errors against the FP64 doubled result per atom;
                and FP64 with a multi-color probe ensemble (one sample, coloring
                radius 6 A) in place of the 256 Rademacher probes; oracle_gate: per
                precision, E, F, gradient blocks and forces of the oracle fixtures' two
                probes against the FP64 oracle (the 1e-6 eV/atom gate)
  overlap       the nonorthogonal basis (S^-1 by conjugate gradients in every step)
                on the 4,000-atom cluster, 200 terms, moments and P, Q blocks
  cluster_steps Chebyshev step throughput on the Cu-like clusters: cu4k in FP64 (4,000
                atoms, 4000 terms, 128 probes) and cu16k in BF16 MFMA (one and two H_hat
                parts), FP32 and FP64
                (16,000 atoms, 8000 terms, 256 probes), moments only, with the HBM and
                arithmetic fractions and the energy errors against FP64 per atom
  copy          a 2 GiB device-to-device copy, timed, as the practical streaming rate
  rational      rational (pole) expansion with CGLS against the Chebyshev expansion
                at matched tolerance on the 4,000-atom cluster (kT = 0.03 eV), both
                with density blocks, errors against a 1e-10 Chebyshev run
"""

import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def acc_updates(p):
    """Steps (of the p - 1) that read and write the density accumulator: the
    library adds the terms of three consecutive steps in one pass, and whatever
    is left at the last step."""
    done, n = 0, 0
    for j in range(1, p):
        if j - done == 3 or j == p - 1:
            done, n = j, n + 1
    return n


def step_bytes(H, s, vt_bytes, mt_bytes, density, p=None):
    bd = H.block_dim
    h = H.nnzb * bd * bd * mt_bytes + H.nnzb * 4 + (H.n_block_rows + 1) * 8
    vec = H.n * s * vt_bytes
    streams = 3.0 + (2.0 * acc_updates(p) / (p - 1) if density else 0.0)
    return h + streams * vec + H.n * s / 8.0


def _code_only(src):
    """Source text without comments and with whitespace collapsed: a digest over it
    changes with the code, not with its comments."""
    src = re.sub(rb"/\*.*?\*/", b" ", src, flags=re.S)
    src = re.sub(rb"//[^\n]*", b" ", src)
    return b" ".join(src.split())


def kernel_digest(read=None):
    """Digest of the step kernel's code: its file, the device helpers and its
    argument struct (the rest of the internal header does not reach the kernel),
    comments left out."""
    csrc = os.path.join(ROOT, "paper_1812_05264_amd", "csrc")
    read = read or (lambda f: open(os.path.join(csrc, f), "rb").read())
    h = hashlib.sha256()
    for f in ("k_step.hip", "device_util.h"):
        h.update(_code_only(read(f)))
    hdr = read("rfo_internal.h")
    i = hdr.index(b"struct StepArgs {")
    h.update(_code_only(hdr[i:hdr.index(b"};", i) + 2]))
    return h.hexdigest()[:16]


def measured_traffic(name):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    e = d.get(name)
    if not e or e.get("kernel_digest") != kernel_digest():
        return None
    return e.get("bytes_per_launch")


def sc64_fp32(H, R, cfg, ref, dens64):
    """The same sc64 call with FP32 vectors and H (FP64 moments, traces and
    coefficients): step time, algorithmic rate and the differences of N, E, F per
    site and of the density blocks against the FP64 call on the same probes."""
    import numpy as np
    import torch
    import paper_1812_05264_amd as pkg
    s, p = cfg.n_probes, cfg.n_terms
    eng = pkg.Engine(0)
    eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 1, H.e_min, H.e_max, "fp32")
    eng.set_probes(R)
    eng.fermi_moments(cfg.T, cfg.mu, p, moments=False, density=True)
    torch.cuda.synchronize()
    eng.set_timing(True)
    g = eng.fermi_moments(cfg.T, cfg.mu, p, moments=False, density=True)
    torch.cuda.synchronize()
    step_ms, n_steps = eng.step_timing()
    eng.set_timing(False)
    eng.close()
    b = step_bytes(H, s, 4, 4, density=True, p=p)
    gbs = b / (step_ms * 1e-3) / 1e9
    d64 = dens64.cpu().numpy()
    out = {"kernel": "k_step1<float, float, 4, 7, 1, true, MODE, false>", "step_us": round(step_ms * 1e3, 2),
           "bytes_per_hv_step": int(b), "GB_per_s": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
           "speedup_vs_fp64_step": None,
           "density_rel_diff": float(np.linalg.norm(g["density"] - d64) / np.linalg.norm(d64))}
    for k in ("N", "E", "F"):
        out[f"d{k}_per_site_vs_fp64"] = abs(g[k] - ref[k]) / H.n
    print(f"[bench] sc64 fp32: step {step_ms * 1e3:.1f} us, {gbs:.0f} GB/s, "
          f"|dN|/site {out['dN_per_site_vs_fp64']:.1e}", flush=True)
    return out


def host_cpu():
    """CPU model and logical CPU count of the host the CPU baseline ran on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def cpu_baseline(H, R, n_steps):
    """The oracle's Chebyshev recurrence (scipy CSR x dense, single-threaded) on the host."""
    import numpy as np
    from oracle import estimator as est
    Hhat = est.mapped_hamiltonian(H)
    t0 = time.perf_counter()
    it = est.chebyshev_vectors(Hhat, R, n_steps + 1)
    for y in it:
        _ = float(np.einsum("ic,ic->", R[:, :1], y[:, :1]))
    dt = time.perf_counter() - t0
    return dt


def oracle_gate(H, cl, cfg, n_terms, precs):
    """The energy+force accuracy gate against the FP64 oracle on its probe subset: the two
    probes of the committed oracle fixtures (tests/golden/oracle_cu16k_grad16.json for the
    per-probe E and F, oracle_cu16k_grad_G.json for the gradient blocks of the 32
    finite-difference atoms' block rows, their forces and F), as a two-probe estimate with
    weights 1/2, in each precision: |F - F_oracle| and |E - E_oracle| per atom, the worst
    per-block relative error of G on those rows, and the force errors on those atoms.
    Returns None when the fixtures are missing or were made for another input."""
    import numpy as np
    import paper_1812_05264_amd as pkg
    from workloads import rademacher
    gold = os.path.join(ROOT, "tests", "golden")
    try:
        fe = json.load(open(os.path.join(gold, "oracle_cu16k_grad16.json")))
        fg = json.load(open(os.path.join(gold, "oracle_cu16k_grad_G.json")))
    except (OSError, ValueError):
        return None
    digest = H.digest()
    if (fe["input_digest"] != digest or fg["input_digest"] != digest or fe["columns"] != fg["columns"]
            or fe["n_terms"] != n_terms or fg["n_terms"] != n_terms):
        return None
    R2 = rademacher(H.n, fe["n_probes_drawn"], config_id=cfg.config_id)[:, fe["columns"]]
    w2 = np.full(R2.shape[1], 1.0 / R2.shape[1])
    scale = w2[0] / fg["weights"][0]
    nz = np.asarray(fg["nz"], dtype=np.int64)
    G_want = scale * np.asarray(fg["G"]).reshape(-1, 9, 9)
    f_want = scale * np.asarray(fg["forces"])
    atoms = np.asarray(fg["atoms"], dtype=np.int64)
    F_want = float(np.dot(w2, fe["F_c"]))
    E_want = float(np.dot(w2, fe["E_c"]))
    D = cl.dH_dR()
    out = {"probes": "the oracle fixtures' two Rademacher probes, weights 1/2",
           "F_oracle_eV": F_want, "E_oracle_eV": E_want}
    for prec in precs:
        eng = pkg.Engine(0)
        eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 9, H.e_min, H.e_max, prec)
        eng.set_probes(R2, w2)
        g = eng.energy_and_dEdH(cfg.T, cfg.mu, n_terms)
        f = eng.hf_forces(D)[atoms]
        eng.close()
        del eng
        Gd = np.max(np.abs(g["dFdH"][nz] - G_want).reshape(nz.size, -1), axis=1)
        Gs = np.max(np.abs(G_want).reshape(nz.size, -1), axis=1)
        r = {"dF_eV_per_atom": abs(g["F"] - F_want) / cl.n_atoms,
             "dE_eV_per_atom": abs(g["E"] - E_want) / cl.n_atoms,
             "G_rows_worst_block_rel_err": float(np.max(Gd / Gs)),
             "force_max_err_eV_per_A": float(np.max(np.abs(f - f_want))),
             "force_rms_err_eV_per_A": float(np.sqrt(np.mean((f - f_want) ** 2)))}
        r["within_1e-6_eV_per_atom"] = bool(r["dF_eV_per_atom"] <= 1e-6 and r["dE_eV_per_atom"] <= 1e-6)
        out[prec] = r
        print(f"[bench] oracle gate {prec}: dF {r['dF_eV_per_atom']:.2e} dE {r['dE_eV_per_atom']:.2e} "
              f"eV/atom, G rows {r['G_rows_worst_block_rel_err']:.2e}, force max "
              f"{r['force_max_err_eV_per_A']:.2e} eV/A", flush=True)
    return out


def energy_force(args):
    import numpy as np
    import paper_1812_05264_amd as pkg
    from workloads.configs import CONFIGS, build_hamiltonian
    from workloads import rademacher
    cfg = CONFIGS["cu16k_grad"]
    H, cl = build_hamiltonian(cfg)
    R = rademacher(H.n, cfg.n_probes, config_id=cfg.config_id)
    D = cl.dH_dR()
    n_terms = args.ef_terms if args.ef_terms > 0 else cfg.n_terms
    out = {"workload": "cu16k_grad", "atoms": cl.n_atoms, "orbitals": H.n, "nnzb": H.nnzb,
           "n_terms": n_terms, "probes": cfg.n_probes, "T_eV": cfg.T, "mu_eV": cfg.mu}
    res = {}
    runs = [(prec, True) for prec in args.ef_precisions.split(",")]
    if args.ef_direct:
        runs.append(("fp64", False))
    import torch
    for prec, doubling in runs:
        eng = pkg.Engine(0)
        eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 9, H.e_min, H.e_max, prec)
        eng.set_probes(R)
        eng.set_moment_doubling(doubling)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = eng.energy_and_dEdH(cfg.T, cfg.mu, n_terms, gradient=False)
        f = eng.hf_forces(D)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        key = prec if doubling else f"{prec}_direct"
        res[key] = (dt, g, f)
        out[f"seconds_{key}"] = round(dt, 4)
        print(f"[bench] energy_force {key}: {dt:.3f} s  F={g['F']:.6f} E={g['E']:.6f}", flush=True)
        eng.close()
        del eng
    if args.ef_colored > 0:
        # multi-color probe ensemble (one sample, weights 1) at coloring radius ef_colored
        from workloads import rademacher_signs
        colours = pkg.welsh_powell(cl.positions, args.ef_colored)
        n_cols = (int(colours.max()) + 1) * 9
        eng = pkg.Engine(0)
        eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 9, H.e_min, H.e_max, "fp64")
        eng.set_colored_probes(colours, 9, rademacher_signs(cl.n_atoms, 9, config_id=cfg.config_id))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = eng.energy_and_dEdH(cfg.T, cfg.mu, n_terms, gradient=False)
        f = eng.hf_forces(D)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        eng.close()
        del eng
        out["colored"] = {"radius_A": args.ef_colored, "colours": int(colours.max()) + 1,
                          "probe_columns": n_cols, "seconds_fp64": round(dt, 4),
                          "F_eV": g["F"]}
        if "fp64" in res:
            _, g64, f64 = res["fp64"]
            out["colored"]["dF_eV_per_atom_vs_rademacher"] = abs(g["F"] - g64["F"]) / cl.n_atoms
            out["colored"]["force_rms_vs_rademacher_eV_per_A"] = float(np.sqrt(np.mean((f - f64) ** 2)))
        print(f"[bench] energy_force colored r={args.ef_colored} ({n_cols} columns): {dt:.3f} s", flush=True)
    if args.ef_gate and n_terms == cfg.n_terms:
        out["oracle_gate"] = oracle_gate(H, cl, cfg, n_terms, args.ef_precisions.split(","))
    if "fp64" in res:
        _, g64, f64 = res["fp64"]
        for prec, (dt, g, f) in res.items():
            if prec == "fp64":
                continue
            out[f"{prec}_vs_fp64"] = {
                "dF_eV_per_atom": abs(g["F"] - g64["F"]) / cl.n_atoms,
                "dE_eV_per_atom": abs(g["E"] - g64["E"]) / cl.n_atoms,
                "force_rms_eV_per_A": float(np.sqrt(np.mean((f - f64) ** 2))),
                "force_max_eV_per_A": float(np.max(np.abs(f - f64))),
            }
    return out


def overlap_leg(args):
    """Nonorthogonal basis: the 4,000-atom Cu-like cluster with the synthetic overlap
    (condition number about 4.5), 128 Rademacher probes, moments and the P and Q
    density blocks over ov_terms terms; every step applies S^-1 by conjugate
    gradients (tolerance 1e-13).  The interval is the rigorous bound
    max|spec H| / lambda_min(S)."""
    import torch
    import paper_1812_05264_amd as pkg
    from workloads import cu_cluster, rademacher
    from workloads.bsr import BSR
    from workloads.overlap import overlap_values, pencil_bound
    cl = cu_cluster(4000, config_id=2)
    H = cl.bsr()
    S = overlap_values(cl)
    a, b = pencil_bound(H, S)
    H = BSR(H.row_ptr, H.col_idx, H.values, 9, a, b)
    R = rademacher(H.n, 128, config_id=2)
    eng = pkg.Engine(0)
    eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 9, a, b, "fp64")
    eng.set_overlap(S, cg_tol=1e-13)
    eng.set_probes(R)
    eng.fermi_moments(0.05, 1.165, 8, density=True)
    it0, so0 = eng.cg_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = eng.fermi_moments(0.05, 1.165, args.ov_terms, density=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    it, so = eng.cg_stats()
    out = {"workload": "cu4k with overlap", "atoms": cl.n_atoms, "probes": 128,
           "n_terms": args.ov_terms, "interval_eV": [round(a, 4), round(b, 4)],
           "seconds": round(dt, 4), "cg_solves": so - so0,
           "cg_iterations_per_solve": round((it - it0) / max(1, so - so0), 2),
           "ms_per_chebyshev_step": round(dt * 1e3 / max(1, args.ov_terms - 1), 3), "N": g["N"]}
    print(f"[bench] overlap cu4k: {dt:.3f} s for {args.ov_terms} terms, "
          f"{out['cg_iterations_per_solve']} CG iterations per solve", flush=True)
    if args.ov_rat_eps > 0:
        out["rational"] = overlap_rational(eng, cl, a, b, args.ov_rat_eps)
    eng.close()
    return out


def overlap_rational(eng, cl, a, b, eps, T=0.05, mu=1.165):
    """Rational against Chebyshev with the overlap at matched tolerance eps: the
    Chebyshev length from the paper's error model on the pencil interval, the
    fewest contour-fit nodes whose error of f on [a, b] is <= eps, CGLS to relative
    residual eps (each CGLS product applies H and S; S^-1 by CG for P, Q)."""
    import numpy as np
    import torch
    import paper_1812_05264_amd as pkg
    p = int(np.ceil(np.log(1.0 / eps) * (b - a) / (6.4 * T)))
    x = np.linspace(a, b, 20001)
    f_exact = 1.0 - np.tanh((x - mu) / (2.0 * T))
    for nodes in range(1, 129):
        fit = pkg.rational_fit(nodes, T, mu, a, b)
        r = fit["f0"] + 2.0 * np.real((1.0 / (x[:, None] - fit["poles"])) @ fit["res_f"])
        if np.max(np.abs(r - f_exact)) <= eps:
            break
    else:
        raise RuntimeError("no fit within 128 nodes")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g_p = eng.fermi_moments(T, mu, p, density=True)
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    it0, _ = eng.rational_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g_r = eng.rational(mu, fit, tol=eps, max_iter=200000, density=True)
    torch.cuda.synchronize()
    t_r = time.perf_counter() - t0
    it1, _ = eng.rational_stats()
    print(f"[bench] overlap cu4k eps={eps:g}: poly {p} terms {t_p:.3f} s, rational "
          f"{2 * nodes} poles {t_r:.3f} s ({it1 - it0} CGLS iterations)", flush=True)
    return {"eps": eps, "poly_terms": p, "poly_s": round(t_p, 4), "rat_poles": 2 * nodes,
            "rat_s": round(t_r, 4), "cgls_iterations": int(it1 - it0),
            "dN_per_atom_rat_vs_poly": abs(g_r["N"] - g_p["N"]) / cl.n_atoms}


PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "bf16x2": 2500.0}


def cluster_steps(args):
    """Step throughput on the Cu-like cluster configurations: cu4k FP64 and cu16k in
    BF16 MFMA (the configuration's precision), FP32 and FP64, one moment-only
    fermi_moments call each (doubled moments: p/2 steps).  Step time from HIP events
    on the library stream; algorithmic bytes per step as for sc64 (H_hat blocks in
    the step's matrix type, columns and row pointers once, three vector streams, probe
    bits); useful flops 2 * 81 * nnzb * s per step against the dense peak of
    the step's arithmetic (FP64, FP32 vector, BF16 MFMA); N, E, F differences per atom
    against the FP64 run on the same probes."""
    import torch
    import paper_1812_05264_amd as pkg
    from workloads.configs import CONFIGS, build_hamiltonian
    from workloads import rademacher
    out = {}
    runs = []
    for item in args.cluster_configs.split(";"):
        if item:
            name, precs = item.split("=")
            runs.append((name, precs.split(",")))
    for name, precs in runs:
        cfg = CONFIGS[name]
        H, cl = build_hamiltonian(cfg)
        s = cfg.n_probes
        R = rademacher(H.n, s, config_id=cfg.config_id)
        rows = {}
        for prec in precs:
            eng = pkg.Engine(0)
            eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 9, H.e_min, H.e_max, prec)
            eng.set_probes(R)
            eng.fermi_moments(cfg.T, cfg.mu, 16, moments=False)
            torch.cuda.synchronize()
            eng.set_timing(True)
            t0 = time.perf_counter()
            n_terms = args.cluster_terms if args.cluster_terms > 0 else cfg.n_terms
            g = eng.fermi_moments(cfg.T, cfg.mu, n_terms, moments=False)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ms, n_steps = eng.step_timing()
            eng.set_timing(False)
            eng.close()
            vt = 8 if prec == "fp64" else 4
            mt = {"fp64": 8, "fp32": 4, "bf16": 2, "bf16x2": 4}[prec]
            b = step_bytes(H, s, vt, mt, density=False)
            flops = 2.0 * 81 * H.nnzb * s
            gbs = b / (ms * 1e-3) / 1e9
            tfs = flops / (ms * 1e-3) / 1e12
            rows[prec] = {"seconds": round(wall, 4), "steps": n_steps, "step_us": round(ms * 1e3, 2),
                          "bytes_per_step": int(b), "GB_per_s": round(gbs, 1),
                          "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "TFLOP_per_s": round(tfs, 2),
                          "frac_compute": round(tfs / PEAK_TFLOPS[prec], 4),
                          "N": g["N"], "E": g["E"], "F": g["F"]}
            print(f"[bench] {name} {prec}: {wall:.3f} s, step {ms * 1e3:.1f} us, {gbs:.0f} GB/s, "
                  f"{tfs:.1f} TFLOP/s", flush=True)
        if "fp64" in rows:
            for prec, r in rows.items():
                if prec != "fp64":
                    for k in ("N", "E", "F"):
                        r[f"d{k}_per_atom_vs_fp64"] = abs(r[k] - rows["fp64"][k]) / cl.n_atoms
        out[name] = {"atoms": cl.n_atoms, "orbitals": H.n, "nnzb": H.nnzb, "probes": s,
                     "n_terms": args.cluster_terms if args.cluster_terms > 0 else cfg.n_terms,
                     "T_eV": cfg.T, "mu_eV": cfg.mu, "runs": rows}
    return out


def copy_bandwidth():
    """Read + write GB/s of a 2 GiB device-to-device copy (the practical streaming rate)."""
    import torch
    n = 256 * 1024 * 1024
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 10
    del x, y
    torch.cuda.empty_cache()
    return 2 * n * 8 / dt / 1e9


def rational_leg(args):
    """Rational against polynomial at matched tolerance eps (the cost comparison of
    the paper's Fig. optimization_fig(b)): the 4,000-atom Cu-like cluster, 128
    Rademacher probes, kT = 0.03 eV, mu = 0, density blocks on.  Chebyshev with
    p = ceil(ln(1/eps) (e_max - e_min) / (6.4 T)) terms (the paper's polynomial
    error model); rational with the fewest contour-fit nodes whose largest error
    of f on [e_min, e_max] is <= eps and CGLS to relative residual eps.  Errors of
    N per atom and of the density blocks are against a Chebyshev run to 1e-10 on
    the same probes, so the probe noise cancels."""
    import numpy as np
    import torch
    import paper_1812_05264_amd as pkg
    from workloads import cu_cluster, rademacher
    cl = cu_cluster(4000, config_id=2)
    H = cl.bsr()
    T, mu = 0.03, 0.0
    R = rademacher(H.n, 128, config_id=2)
    eng = pkg.Engine(0)
    eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 9, H.e_min, H.e_max, "fp64")
    eng.set_probes(R)
    width = H.e_max - H.e_min
    p_of = lambda eps: int(np.ceil(np.log(1.0 / eps) * width / (6.4 * T)))
    ref = eng.fermi_moments(T, mu, p_of(1e-10), moments=False, density=True)
    x = np.linspace(H.e_min, H.e_max, 20001)
    f_exact = 1.0 - np.tanh((x - mu) / (2.0 * T))

    def fit_for(eps):
        for n in range(1, 129):
            fit = pkg.rational_fit(n, T, mu, H.e_min, H.e_max)
            r = fit["f0"] + 2.0 * np.real((1.0 / (x[:, None] - fit["poles"])) @ fit["res_f"])
            if np.max(np.abs(r - f_exact)) <= eps:
                return n, fit
        raise RuntimeError("no fit within 128 nodes")

    eng.rational(mu, pkg.rational_fit(1, T, mu, H.e_min, H.e_max), tol=1e-2, density=True)
    rows = []
    for eps in [float(e) for e in args.rat_eps.split(",") if e]:
        p = p_of(eps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g_p = eng.fermi_moments(T, mu, p, moments=False, density=True)
        torch.cuda.synchronize()
        t_p = time.perf_counter() - t0
        nodes, fit = fit_for(eps)
        it0, so0 = eng.rational_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g_r = eng.rational(mu, fit, tol=eps, max_iter=200000, density=True)
        torch.cuda.synchronize()
        t_r = time.perf_counter() - t0
        it1, so1 = eng.rational_stats()
        dref = np.linalg.norm(ref["density"])
        rows.append({
            "eps": eps, "poly_terms": p, "poly_s": round(t_p, 4),
            "rat_nodes": nodes, "rat_poles": 2 * nodes, "rat_s": round(t_r, 4),
            "cgls_iterations": int(it1 - it0), "cgls_iterations_max_pole": int(np.max(g_r["iterations"])),
            "poly_dN_per_atom": abs(g_p["N"] - ref["N"]) / cl.n_atoms,
            "rat_dN_per_atom": abs(g_r["N"] - ref["N"]) / cl.n_atoms,
            "poly_density_rel_err": float(np.linalg.norm(g_p["density"] - ref["density"]) / dref),
            "rat_density_rel_err": float(np.linalg.norm(g_r["density"] - ref["density"]) / dref),
        })
        print(f"[bench] rational cu4k eps={eps:g}: poly {p} terms {t_p:.3f} s, rational "
              f"{2 * nodes} poles {t_r:.3f} s ({it1 - it0} CGLS iterations)", flush=True)
    eng.close()
    return {"workload": "cu4k: 4,000-atom Cu-like cluster, 128 Rademacher probes, kT=0.03 eV, "
                        "mu=0, density blocks", "atoms": cl.n_atoms, "points": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--cpu-steps", type=int, default=80,
                    help="oracle Chebyshev steps timed for the CPU baseline (0 = skip)")
    ap.add_argument("--energy-force", type=int, default=1)
    ap.add_argument("--ef-precisions", default="fp64,fp32,bf16,bf16x2")
    ap.add_argument("--ef-direct", type=int, default=1,
                    help="also time FP64 energy_force with the direct recurrence (no doubling)")
    ap.add_argument("--ef-gate", type=int, default=1,
                    help="energy_force: errors against the FP64 oracle fixtures per precision (0 = skip)")
    ap.add_argument("--ef-colored", type=float, default=6.0,
                    help="coloring radius (A) of a multi-color probe energy_force run (0 = skip)")
    ap.add_argument("--ov-terms", type=int, default=200,
                    help="terms of the overlap (nonorthogonal basis) leg (0 = skip)")
    ap.add_argument("--ov-rat-eps", type=float, default=1e-3,
                    help="overlap leg: rational vs Chebyshev at this tolerance (0: off)")
    ap.add_argument("--cluster-steps", type=int, default=1,
                    help="step throughput legs on the Cu-like clusters (0 = skip)")
    ap.add_argument("--rat-eps", default="1e-3",
                    help="tolerances of the rational-vs-polynomial leg (empty = skip)")
    ap.add_argument("--ef-terms", type=int, default=0,
                    help="Chebyshev terms of the energy_force leg (0 = the workload's 8000)")
    ap.add_argument("--only-energy-force", action="store_true",
                    help="run only the energy_force leg (for profiling)")
    ap.add_argument("--sc64-fp32", type=int, default=1,
                    help="also time sc64 with FP32 steps and report its differences (0 = skip)")
    ap.add_argument("--cluster-configs", default="cu4k=fp64;cu16k=bf16,bf16x2,fp32,fp64",
                    help="cluster step legs: config=precisions, separated by ';'")
    ap.add_argument("--cluster-terms", type=int, default=0,
                    help="Chebyshev terms of the cluster step legs (0 = the configuration's)")
    ap.add_argument("--only-cluster", action="store_true",
                    help="run only the cluster step legs (for profiling)")
    ap.add_argument("--only-overlap", action="store_true",
                    help="run only the overlap leg")
    ap.add_argument("--only-rational", action="store_true",
                    help="run only the rational-vs-polynomial leg (for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="time a 2 GiB device-to-device copy (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the hot path is measured on one GPU's share of "
              "the probes; runs on several GPUs are not implemented", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        import torch
        n = 256 * 1024 * 1024
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            y.copy_(x)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 10
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8,
                          "GB_per_s_read_plus_write": round(2 * n * 8 / dt / 1e9, 1)}))
        return
    if args.only_energy_force:
        print(json.dumps({"energy_force": energy_force(args)}))
        return
    if args.only_rational:
        print(json.dumps({"rational": rational_leg(args)}))
        return
    if args.only_overlap:
        print(json.dumps({"overlap": overlap_leg(args)}))
        return
    if args.only_cluster:
        print(json.dumps({"cluster_steps": cluster_steps(args)}))
        return

    import numpy as np
    import torch
    import paper_1812_05264_amd as pkg
    from workloads.configs import CONFIGS, build_hamiltonian
    from workloads import rademacher

    cfg = CONFIGS["sc64"]
    H, _ = build_hamiltonian(cfg)
    s, p = cfg.n_probes, cfg.n_terms
    R = rademacher(H.n, s, config_id=cfg.config_id)
    eng = pkg.Engine(0)
    eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 1, H.e_min, H.e_max, args.precision)
    eng.set_probes(R)
    vt = 8 if args.precision == "fp64" else 4
    b_step = step_bytes(H, s, vt, vt, density=True, p=p)
    dens = torch.empty((H.nnzb, 1, 1), dtype=torch.float64, device="cuda")

    for _ in range(args.warmup):
        eng.fermi_moments(cfg.T, cfg.mu, p, moments=False, density_out=dens)
    torch.cuda.synchronize()
    eng.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for _ in range(args.steps):
        last = eng.fermi_moments(cfg.T, cfg.mu, p, moments=False, density_out=dens)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms, n_steps = eng.step_timing()
    eng.set_timing(False)
    total_bytes = b_step * (p - 1) * args.steps
    value = total_bytes / wall / 1e9
    achieved = b_step / (step_ms * 1e-3) / 1e9
    # the step kernel is launched as two variants: MODE 1 on the steps that
    # update the density accumulator, MODE 0 on the others (7 neighbours per
    # chunk: every row of the lattice has 7 entries)
    kname = ("k_step1<double, double, 2, 7, 1, true, MODE, false>" if args.precision == "fp64"
             else "k_step1<float, float, 4, 7, 1, true, MODE, false>")
    traffic = measured_traffic("sc64_" + args.precision)
    print(f"[bench] sc64 {args.precision}: {wall / args.steps * 1e3:.1f} ms per call, step kernel "
          f"{step_ms * 1e3:.1f} us ({n_steps} steps), {achieved:.0f} GB/s, N={last['N']:.6f}",
          flush=True)

    line = {
        "metric": "Chebyshev H.V step GB/s (frac HBM peak); energy+force time at 1e-6 eV/atom",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "chebyshev_steps_per_step": p - 1,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "sc64: simple-cubic L=64 (262144 sites), t=-1, onsite U[-0.5,0.5], "
                               "kT=0.02, mu=0.3, 2048 Chebyshev terms, 256 Rademacher probes, "
                               "density blocks on",
                   "sites": H.n, "nnz": H.nnzb, "probes": s, "n_terms": p,
                   "bytes_per_hv_step": int(b_step)},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "mean_launch_us": round(step_ms * 1e3, 2)},
    }
    # the same achieved rate against what a plain device copy moves on this GPU
    cb = copy_bandwidth()
    line["roofline"]["copy_GBps"] = round(cb, 1)
    line["roofline"]["frac_of_copy"] = round(achieved / cb, 4)

    if args.cpu_steps > 0:
        n_sample = args.cpu_steps
        dt = cpu_baseline(H, R, n_sample)
        b_cpu = step_bytes(H, s, 8, 8, density=False)
        line["cpu_baseline"] = {"value": round(b_cpu * n_sample / dt / 1e9, 4), "unit": "GB/s",
                                "cores": 1, "kind": "oracle",
                                "sample": f"{n_sample} Chebyshev steps of the FP64 oracle (scipy CSR "
                                          f"x dense, single-threaded) on sc64 with all {s} probes; "
                                          f"{dt:.1f} s",
                                "host": host_cpu()}
    if args.sc64_fp32 and args.precision == "fp64":
        line["sc64_fp32"] = sc64_fp32(H, R, cfg, last, dens)
        line["sc64_fp32"]["speedup_vs_fp64_step"] = round(step_ms / (line["sc64_fp32"]["step_us"] * 1e-3), 3)
    if args.energy_force:
        eng.close()
        del eng
        torch.cuda.empty_cache()
        line["energy_force"] = energy_force(args)
    if args.ov_terms > 0:
        torch.cuda.empty_cache()
        line["overlap"] = overlap_leg(args)
    if args.cluster_steps:
        torch.cuda.empty_cache()
        line["cluster_steps"] = cluster_steps(args)
    if args.rat_eps:
        torch.cuda.empty_cache()
        line["rational"] = rational_leg(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
