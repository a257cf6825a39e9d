"""Executed matrix-core flops and matrix-core busy time per kernel family,
from one rocprofv3 counter run.

The run (OUT is any output directory; default kernel shapes, so no autotuner
launches; one reduced C2 step of 16 E x 8 k points):

    rocprofv3 --pmc SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_VALU_MFMA_BUSY_CYCLES \
        GRBM_GUI_ACTIVE -d OUT/pmc_mfma -o run -- python3 bench.py --n-e 16 --no-cpu-baseline \
        --tune default > OUT/pmc_mfma.log

SQ_INSTS_VALU_MFMA_MOPS_* counts matrix-core work in units of 512 flops, so
the executed flops of a dispatch are 512 x that count.  The busy share is
SQ_VALU_MFMA_BUSY_CYCLES over (active cycles x SIMDs), the counter tool's own
MfmaUtil; the active cycles are GRBM_GUI_ACTIVE of one XCD (the counter comes
back summed over the eight).  For the batched GEMM the executed flops are set against the
algorithmic 8 b^3 per point-launch the bench line counts: with complex products
as three real products the ratio is 3/4.
Writes profiles/mfma_counters_C2.md.  Usage: python profile_mfma.py OUT
"""
import collections
import json
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
SIMDS = 256 * 4
XCDS = 8   # GRBM_GUI_ACTIVE comes back summed over the eight XCDs' instances
COUNTERS = ("SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_VALU_MFMA_BUSY_CYCLES",
            "GRBM_GUI_ACTIVE")


def family(name):
    for key, fam in (("gemm_kernel", "batched GEMM"), ("gemm_persist", "batched GEMM"), ("gj_update", "inverse update"),
                     ("gj_panel", "inverse panel")):
        if key in name:
            return fam
    return "other"


def main(base):
    out_dir = os.path.basename(os.path.normpath(base))
    db = sqlite3.connect(os.path.join(base, "pmc_mfma", "run_results.db"))
    rows = db.execute("select dispatch_id, kernel_name, counter_name, sum(value) from counters_collection "
                      "group by dispatch_id, counter_name").fetchall()
    disp = collections.defaultdict(dict)
    names = {}
    for d, k, c, v in rows:
        disp[d][c] = v
        names[d] = k
    agg = collections.defaultdict(lambda: collections.Counter())
    for d, cs in disp.items():
        a = agg[family(names[d])]
        a["dispatches"] += 1
        for c in COUNTERS:
            a[c] += cs.get(c, 0.0)
    with open(os.path.join(base, "pmc_mfma.log")) as fh:
        bench = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    r = bench["roofline"]
    b = bench["config"]["block"]
    gemm_alg = 8.0 * b ** 3 * r["points_per_launch"] * r["launches"]
    g = agg["batched GEMM"]
    assert g["dispatches"] == r["launches"], (g["dispatches"], r["launches"])
    lines = [
        f"# Executed matrix-core flops per kernel family, C2 block {b}, {bench['config']['slabs']} slabs, "
        f"{bench['config']['n_e']} E x {bench['config']['n_k']} k (FP64), MI355X",
        "",
        "Command (run from /tmp with TMPDIR=/tmp; one counter pass, default kernel shapes):",
        "",
        "    rocprofv3 --pmc " + " ".join(COUNTERS) + f" -d {out_dir}/pmc_mfma -o run -- \\",
        f"        python3 bench.py --n-e 16 --no-cpu-baseline --tune default > {out_dir}/pmc_mfma.log",
        f"    python profile_mfma.py {out_dir}",
        "",
        "Executed flops = 512 x SQ_INSTS_VALU_MFMA_MOPS_*; matrix-core busy = SQ_VALU_MFMA_BUSY_CYCLES / "
        f"(GRBM_GUI_ACTIVE / {XCDS} XCDs x {SIMDS} SIMDs), summed over the family's dispatches (counters "
        "serialise dispatches). The busy counter advances 16 cycles per 512 FP64 matrix-core flops (one "
        "v_mfma_f64_16x16x4f64 = 4 units, 64 cycles), so the busy share is the executed rate over the peak rate "
        "at the clock the kernels ran at.",
        "",
        "| family | dispatches | executed FP64 MFMA flops | executed FP32 MFMA flops | matrix cores busy |",
        "|---|---|---|---|---|",
    ]
    for fam in ("batched GEMM", "inverse update", "inverse panel", "other"):
        a = agg.get(fam)
        if not a:
            continue
        busy = a["SQ_VALU_MFMA_BUSY_CYCLES"] / (a["GRBM_GUI_ACTIVE"] / XCDS * SIMDS) if a["GRBM_GUI_ACTIVE"] else 0.0
        lines.append(f"| {fam} | {a['dispatches']} | {512 * a['SQ_INSTS_VALU_MFMA_MOPS_F64']:.4e} | "
                     f"{512 * a['SQ_INSTS_VALU_MFMA_MOPS_F32']:.4e} | {100 * busy:.1f} % |")
    ex = 512 * g["SQ_INSTS_VALU_MFMA_MOPS_F64"]
    lines += [
        "",
        f"Batched GEMM: {g['dispatches']} dispatches (the bench line's timed launches: {r['launches']}), "
        f"{r['points_per_launch']:.1f} full-product points per launch; algorithmic 8 b^3 per point-launch = "
        f"{gemm_alg:.4e} flops; executed on matrix cores {ex:.4e} flops; executed / algorithmic = "
        f"{ex / gemm_alg:.4f} (3M form: 0.75).",
    ]
    with open(os.path.join(ROOT, "profiles", "mfma_counters_C2.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if len(sys.argv) != 2:
        sys.exit("usage: python profile_mfma.py OUT  (the directory the rocprofv3 run wrote into)")
    main(sys.argv[1])
