"""HBM traffic of the batched GEMM from two rocprofv3 counter runs.

Reads the FETCH_SIZE and WRITE_SIZE databases that these commands write into
an output directory OUT (one counter per run, each run also copies a known
256 MiB buffer first so the counters can be calibrated; both use the library's
default kernel shapes so the two runs dispatch the same kernels):

    rocprofv3 --pmc FETCH_SIZE -d OUT/pmc_FETCH_SIZE -o run -- \
        python3 bench.py --n-e 16 --no-cpu-baseline --tune default --copy-calibration 256 > OUT/pmc_FETCH_SIZE.log
    rocprofv3 --pmc WRITE_SIZE -d OUT/pmc_WRITE_SIZE -o run -- \
        python3 bench.py --n-e 16 --no-cpu-baseline --tune default --copy-calibration 256 > OUT/pmc_WRITE_SIZE.log

and writes profiles/gemm_traffic_C2.json (read by bench.py for the roofline's
`traffic`, valid while the GEMM sources keep the recorded SHA-1) and a short
text summary that records the commands with OUT as given.
Usage: python profile_traffic.py OUT
"""
import collections
import hashlib
import json
import os
import re
import sqlite3
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
GEMM_SOURCES = ["negf_gemm.hip", "negf_mfma.hpp", "negf_common.hpp", "negf_internal.hpp"]
COPY_BYTES = 256 << 20


def _rows(base, counter):
    db = sqlite3.connect(os.path.join(base, f"pmc_{counter}", "run_results.db"))
    return db.execute("select dispatch_id, kernel_name, grid_size, value from counters_collection "
                      "order by dispatch_id").fetchall()


def _bench_line(base, counter):
    with open(os.path.join(base, f"pmc_{counter}.log")) as fh:
        return json.loads([ln for ln in fh if ln.startswith("{")][-1])


def sources_sha1():
    h = hashlib.sha1()
    for f in GEMM_SOURCES:
        with open(os.path.join(ROOT, "paper_1510_04686_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def main(base):
    out_dir = os.path.basename(os.path.normpath(base))
    fetch, write = _rows(base, "FETCH_SIZE"), _rows(base, "WRITE_SIZE")
    assert [r[1] for r in fetch] == [r[1] for r in write], "the two runs dispatched different kernels"
    copy_f = [v for _, k, g, v in fetch if "copyBuffer" in k and g == 131072][0] * 1024
    copy_w = [v for _, k, g, v in write if "copyBuffer" in k and g == 131072][0] * 1024
    ff, fw = COPY_BYTES / copy_f, COPY_BYTES / copy_w
    gemm_f = sum(v for _, k, _, v in fetch if "gemm_kernel" in k) * 1024 * ff
    gemm_w = sum(v for _, k, _, v in write if "gemm_kernel" in k) * 1024 * fw
    n_disp = sum(1 for _, k, _, _ in fetch if "gemm_kernel" in k)
    bench = _bench_line(base, "FETCH_SIZE")
    b = bench["config"]["block"]
    roof = bench["roofline"]
    # full-product-equivalent point launches (the anti-Hermitian launches count the
    # share of tiles they compute), as bench.py counts them
    point_launches = roof["launches"] * roof["points_per_launch"]
    per_pl = (gemm_f + gemm_w) / point_launches
    out = {
        "kernel": "negf::gemm_kernel (all epilogue/op instantiations), FP64",
        "workload": f"C2 block {b}, {bench['config']['slabs']} slabs, {bench['config']['n_e']} E x "
                    f"{bench['config']['n_k']} k ({bench['config']['batch_capacity']} points per launch)",
        "kernel_sources_sha1": sources_sha1(),
        "gemm_dispatches": n_disp,
        "point_launches": point_launches,
        "fetch_bytes_calibrated": gemm_f,
        "write_bytes_calibrated": gemm_w,
        "hbm_bytes_per_point_launch": per_pl,
        "algorithmic_bytes_per_point_launch": 3 * 16 * b * b,
        "calibration": {"copy_bytes": COPY_BYTES, "FETCH_SIZE_factor": ff, "WRITE_SIZE_factor": fw},
        "commands": [
            f"rocprofv3 --pmc {c} -d {out_dir}/pmc_{c} -o run -- python3 bench.py --n-e 16 "
            "--no-cpu-baseline --tune default --copy-calibration 256"
            for c in ("FETCH_SIZE", "WRITE_SIZE")
        ],
    }
    with open(os.path.join(ROOT, "profiles", "gemm_traffic_C2.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    agg = collections.defaultdict(lambda: [0, 0.0, 0.0])
    for (_, k, _, vf), (_, _, _, vw) in zip(fetch, write):
        name = re.sub(r"HIP_vector_type<(double|float), 2u>", lambda m: "c128" if m.group(1) == "double" else "c64",
                      k).split("(")[0][:90]
        a = agg[name]
        a[0] += 1
        a[1] += vf
        a[2] += vw
    lines = [
        f"# HBM traffic of the batched complex GEMM (and neighbours), {out['workload']}",
        "",
        "Commands (one counter per run, each with one plain 256 MiB device copy first for calibration):",
        "",
        *["    " + c for c in out["commands"]],
        f"    python profile_traffic.py {out_dir}",
        "",
        f"Calibration (the 256 MiB copy): FETCH_SIZE factor {ff:.2f}, WRITE_SIZE factor {fw:.2f}.",
        "",
        f"GEMM family ({n_disp} dispatches, {point_launches:,.0f} full-product point-launches): calibrated "
        f"{gemm_f / 1e9:.1f} GB fetched + {gemm_w / 1e9:.1f} GB written = {per_pl / 1e6:.2f} MB per point-launch, "
        f"against {3 * 16 * b * b / 1e6:.2f} MB algorithmic (read A, B; write C) -> "
        f"{per_pl / (3 * 16 * b * b):.2f}x.",
        "",
        "Raw per-dispatch averages (MiB, uncalibrated FETCH_SIZE / WRITE_SIZE):",
        "",
        "```",
    ]
    for name, (n, f, w) in sorted(agg.items(), key=lambda x: -x[1][1])[:16]:
        lines.append(f"{n:6d} fetch {f / n / 1024:9.2f} MiB/disp  write {w / n / 1024:9.2f} MiB/disp  {name}")
    lines.append("```")
    with open(os.path.join(ROOT, "profiles", "gemm_traffic_C2.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    if len(sys.argv) != 2:
        sys.exit("usage: python profile_traffic.py OUT  (the directory the two rocprofv3 runs wrote into)")
    main(sys.argv[1])
