"""Profiling helpers for the IRE tracer.

    python -m paper_2408_13807_amd.profiling valu-cases OUT.json
        one-lane FP32 runs of several clouds (run it under
        `rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_WAVES`);
        writes their event counts in dispatch order
    python -m paper_2408_13807_amd.profiling valu-fit DB OUT.json
        least-squares fit of SQ_INSTS_VALU = c0 + sum_e c_e n_e over those
        dispatches: the VALU instructions one lane executes per event type
    python -m paper_2408_13807_amd.profiling summary DB [DB ...]
        markdown summary of rocprofv3 databases (kernel statistics and counters)
    python -m paper_2408_13807_amd.profiling copy [MiB]
        one device-to-device copy of MiB (default 1024) MiB: the reference
        dispatch that scales FETCH_SIZE / WRITE_SIZE into bytes
    python -m paper_2408_13807_amd.profiling sur-predict [rows]
        surrogate ensemble prediction (5 members, 4 x 256) of `rows` (default
        2.1e7) device-resident rows, three launches: the MFMA kernel to profile
    python -m paper_2408_13807_amd.profiling valu-rate
        lane-operations per second of plain FP32 FMAs and adds, hardware
        transcendentals and 32-bit high multiplies (csrc/valu_rate.hip): the
        measured side of the VALU peak
    python -m paper_2408_13807_amd.profiling sur-train [steps]
        `steps` (default 200) training steps of the same ensemble on random
        rows, 4096 per member and step: the forward, backward and weight-gradient
        MFMA kernels to profile
"""
from __future__ import annotations

import json
import sqlite3
import sys

import numpy as np

EVENTS = ("n_cross", "n_launch", "n_scat", "n_abs")
FLIGHT_EVENTS = ("n_launch", "n_scat", "n_abs")


def valu_cases() -> list[dict]:
    from paper_2408_13807_amd import ire, workloads as wl
    scat = dict(wl.cfg_external_small())
    scat["albedo"] = np.full(64, 0.9)
    cases = [("ext50", wl.cfg_external_small(), dict(n_ext=2000)),
             ("ext101", wl.cfg_external_large(), dict(n_ext=1000)),
             ("central200", wl.cfg_central(), dict(n_ps=200)),
             ("gray_abs", wl.gray_model(20, 5.0, external=True), dict(n_ext=2000)),
             ("scat_heavy", scat, dict(n_ext=500)),
             ("ext50_short", wl.cfg_external_small(), dict(n_ext=200))]
    out = []
    for name, m, kw in cases:
        # one package in flight and one atomic per absorption: no grouping code,
        # and the workgroup's idle waves run no event passes beside it (their
        # instructions are no work of the package)
        r = ire.run_model(m, seed=1, max_lanes=1, aggregate=0, **kw)
        out.append(dict(name=name, **{k: r["stats"][k] for k in EVENTS + ("n_step_slots",)}))
    return out


def _counters(db: str) -> list[dict]:
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection "
                       "order by dispatch_id").fetchall()
    per = {}
    names = {}
    for d, k, c, v in rows:
        per.setdefault(d, {})[c] = v
        names[d] = k
    return [dict(kernel=names[d], **per[d]) for d in sorted(per)]


def valu_fit(db: str, cases: list[dict]) -> dict:
    """Least squares SQ_INSTS_VALU = c0 + c_step * steps + sum_e c_e n_e over
    the one-lane runs, steps = the lane's crossing-sweep steps (n_step_slots /
    64).  A sweep runs several steps per check, so after its lane parks a
    sweep may run a few steps that move nothing: fitting the steps apart from
    the events keeps those out of the events' costs.  The algorithmic work of
    an event is then its own path plus the one step that found it (every event
    but an escape ends a flight), and of a crossing one step."""
    disp = [c for c in _counters(db) if "ire_trace" in c["kernel"]]
    if len(disp) != len(cases):
        raise ValueError(f"{len(disp)} tracer dispatches but {len(cases)} cases")
    X = np.array([[1.0, c["n_step_slots"] / 64.0] + [c[e] for e in FLIGHT_EVENTS] for c in cases])
    y = np.array([d["SQ_INSTS_VALU"] for d in disp])
    coef = np.linalg.lstsq(X, y, rcond=None)[0]
    resid = (X @ coef - y) / y
    c_step = float(coef[1])
    return {"per_lane_valu": {"step": c_step, **{e[2:]: float(c) for e, c in zip(FLIGHT_EVENTS, coef[2:])}},
            "algorithmic_per_event": {"cross": c_step,
                                      **{e[2:]: float(c) + c_step for e, c in zip(FLIGHT_EVENTS, coef[2:])}},
            "constant": float(coef[0]), "max_rel_residual": float(np.max(np.abs(resid))),
            "cases": [dict(c, SQ_INSTS_VALU=d["SQ_INSTS_VALU"]) for c, d in zip(cases, disp)]}


def summary(dbs: list[str]) -> str:
    lines = []
    for db in dbs:
        con = sqlite3.connect(db)
        lines.append(f"### {db}\n")
        try:
            rows = con.execute("select name, total_calls, total_duration, average, percentage "
                               "from top_kernels").fetchall()
        except sqlite3.Error:
            rows = []
        if rows:
            lines.append("| kernel | calls | total (ms) | average (ms) | % |")
            lines.append("|---|---|---|---|---|")
            for name, calls, tot, avg, pct in rows:
                lines.append(f"| `{name[:90]}` | {calls} | {tot / 1e3:.3f} | {avg / 1e3:.4f} | {pct:.2f} |")
            lines.append("")
        cnt = _counters(db)
        if cnt:
            keys = sorted({k for c in cnt for k in c if k != "kernel"})
            lines.append("| dispatch kernel | " + " | ".join(keys) + " |")
            lines.append("|---|" + "---|" * len(keys))
            for c in cnt:
                if not any(k in c["kernel"] for k in ("ire_", "sur_", "copy", "Copy")):
                    continue
                lines.append(f"| `{c['kernel'][:60]}` | " + " | ".join(f"{c.get(k, float('nan')):.6g}" for k in keys) + " |")
            lines.append("")
    return "\n".join(lines)


def main(argv: list[str]) -> int:
    if not argv:
        print(__doc__)
        return 1
    cmd = argv[0]
    if cmd == "valu-cases":
        res = valu_cases()
        with open(argv[1], "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res))
    elif cmd == "valu-fit":
        with open(argv[2]) as f:
            cases = json.load(f)
        print(json.dumps(valu_fit(argv[1], cases), indent=1))
    elif cmd == "summary":
        print(summary(argv[1:]))
    elif cmd == "sur-predict":
        import time
        import torch
        from paper_2408_13807_amd import surrogate
        n = int(float(argv[1])) if len(argv) > 1 else 21_000_000
        rng = np.random.default_rng(0)
        net = surrogate.SurNet(members=5, depth=4, seed=1)
        net.set_normalization(np.zeros(6), np.ones(6), 1.3, 0.3)
        X = torch.from_numpy(rng.normal(size=(n, 6)).astype(np.float32)).cuda()
        mean = torch.empty(n, device="cuda")
        spread = torch.empty(n, device="cuda")
        torch.cuda.synchronize()
        for _ in range(3):
            t0 = time.perf_counter()
            net.predict_dev(X.data_ptr(), n, mean.data_ptr(), spread.data_ptr())
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            # dense FLOPs of the network's 7 inputs (the input tile is padded to 32 for the MFMA)
            flop = 2.0 * n * 5 * (7 * 256 + 3 * 256 * 256 + 256)
            print(json.dumps({"rows": n, "s": dt, "rows_per_s": n / dt, "tflops": flop / dt / 1e12}), flush=True)
        net.close()
    elif cmd == "sur-train":
        # training steps of a 5-member ensemble on random rows (4096 rows per member and step)
        import time
        import torch
        from paper_2408_13807_amd import surrogate
        steps = int(argv[1]) if len(argv) > 1 else 200
        rng = np.random.default_rng(0)
        X = rng.normal(size=(1 << 20, 6)).astype(np.float32)
        y = (1.3 + 0.3 * np.tanh(X[:, 0]) + 0.1 * X[:, 5]).astype(np.float32)
        net = surrogate.SurNet(members=5, depth=4, seed=1)
        net.set_normalization(np.zeros(6), np.ones(6), 1.3, 0.3)
        net.train(X, y, steps=4, batch=4096)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = net.train(X, y, steps=steps, batch=4096)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # forward, backward and weight gradient: 3x the forward FLOPs of 5 x 4096 rows per step
        flop = 3 * 2.0 * 4096 * 5 * (7 * 256 + 3 * 256 * 256 + 256) * steps
        print(json.dumps({"steps": steps, "s": dt, "steps_per_s": steps / dt, "tflops": flop / dt / 1e12,
                          "loss": [float(v) for v in loss]}), flush=True)
        net.close()
    elif cmd == "valu-rate":
        import os
        import subprocess
        from paper_2408_13807_amd import build
        if not os.path.exists(build.VALU_RATE):
            raise SystemExit(f"{build.VALU_RATE} is not built; run __graft_entry__.build()")
        print(subprocess.run([build.VALU_RATE], check=True, capture_output=True, text=True).stdout, end="")
    elif cmd == "copy":
        import torch
        n = (int(argv[1]) if len(argv) > 1 else 1024) << 18   # float32 elements
        x = torch.ones(n, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}))
    else:
        print(__doc__)
        return 1
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
