"""Where the waves of the main kernel families spend their cycles, from
two rocprofv3 counter passes on the reduced C2 command (default kernel shapes):

    rocprofv3 --pmc SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_WAIT_INST_LDS SQ_ACTIVE_INST_ANY \
        SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_VMEM SQ_ACTIVE_INST_VALU -d OUT/pmc_stall1 -o run -- \
        python3 bench.py --n-e 16 --no-cpu-baseline --tune default
    rocprofv3 --pmc SQ_BUSY_CYCLES SQ_LDS_IDX_ACTIVE SQ_LDS_BANK_CONFLICT SQ_LDS_DATA_FIFO_FULL \
        SQ_LDS_CMD_FIFO_FULL SQ_INSTS_LDS SQ_INSTS_VALU SQ_INSTS_MFMA -d OUT/pmc_stall2 -o run -- \
        python3 bench.py --n-e 16 --no-cpu-baseline --tune default

The SQ_WAIT_* and SQ_ACTIVE_INST_* counters are cycles summed over waves, so
each is shown as a share of SQ_WAVE_CYCLES (the cycles waves were resident):
waiting on a dependency (a memory or LDS result, a barrier), waiting for an
issue slot, and issuing LDS, memory or vector instructions.  The LDS counters
are shown against SQ_BUSY_CYCLES.  Writes profiles/stalls_C2.md.
Usage: python profile_stalls.py OUT
"""
import collections
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
PASS1 = ("SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS", "SQ_ACTIVE_INST_ANY",
         "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_VMEM", "SQ_ACTIVE_INST_VALU")
PASS2 = ("SQ_BUSY_CYCLES", "SQ_LDS_IDX_ACTIVE", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_DATA_FIFO_FULL",
         "SQ_LDS_CMD_FIFO_FULL", "SQ_INSTS_LDS", "SQ_INSTS_VALU", "SQ_INSTS_MFMA")
FAMILIES = (("gemm_kernel", "batched GEMM"), ("gemm_persist", "batched GEMM"), ("gj_update", "inverse update"),
            ("gj_panel", "inverse panel"), ("sandwich", "coupling sandwich"), ("bond_rows", "bond trace"))


def family(name):
    for key, fam in FAMILIES:
        if key in name:
            return fam
    return None


def totals(path):
    db = sqlite3.connect(path)
    agg = collections.defaultdict(collections.Counter)
    for k, c, v in db.execute("select kernel_name, counter_name, sum(value) from counters_collection "
                              "group by dispatch_id, counter_name"):
        f = family(k)
        if f:
            agg[f][c] += v
    return agg


def main(base):
    out_dir = os.path.basename(os.path.normpath(base))
    p1 = totals(os.path.join(base, "pmc_stall1", "run_results.db"))
    p2 = totals(os.path.join(base, "pmc_stall2", "run_results.db"))
    order = ["batched GEMM", "inverse update", "inverse panel", "coupling sandwich", "bond trace"]
    lines = [
        "# Wave-cycle breakdown of the kernel families, reduced C2 (block 400, 70 slabs, 16 E x 8 k, FP64), MI355X",
        "",
        "Commands (run from /tmp with TMPDIR=/tmp; two counter passes, default kernel shapes):",
        "",
        "    rocprofv3 --pmc " + " ".join(PASS1) + f" -d {out_dir}/pmc_stall1 -o run -- \\",
        "        python3 bench.py --n-e 16 --no-cpu-baseline --tune default",
        "    rocprofv3 --pmc " + " ".join(PASS2) + f" -d {out_dir}/pmc_stall2 -o run -- \\",
        "        python3 bench.py --n-e 16 --no-cpu-baseline --tune default",
        f"    python profile_stalls.py {out_dir}",
        "",
        "Shares of SQ_WAVE_CYCLES (cycles summed over resident waves): waiting on a dependency (SQ_WAIT_ANY), "
        "waiting for an issue slot (SQ_WAIT_INST_ANY; of it, behind LDS: SQ_WAIT_INST_LDS), issuing any "
        "instruction, LDS, vector-memory and VALU instructions (SQ_ACTIVE_INST_*).",
        "",
        "| family | wait dependency | wait issue | wait issue (LDS) | issuing any | LDS | VMEM | VALU |",
        "|---|---|---|---|---|---|---|---|",
    ]
    for f in order:
        a = p1.get(f)
        if not a or not a["SQ_WAVE_CYCLES"]:
            continue
        w = a["SQ_WAVE_CYCLES"]
        cols = [a[c] / w for c in PASS1[1:]]
        lines.append(f"| {f} | " + " | ".join(f"{100 * x:.1f} %" for x in cols) + " |")
    lines += [
        "",
        "LDS pressure relative to SQ_BUSY_CYCLES: cycles the LDS was active (SQ_LDS_IDX_ACTIVE), bank-conflict "
        "cycles, cycles its data and command FIFOs were full. Both sides are summed over counter instances, so "
        "these ratios compare the families rather than give an occupancy. Then the instruction mix (LDS, VALU "
        "and MFMA instructions, per-SE totals).",
        "",
        "| family | LDS active | bank conflict | data FIFO full | command FIFO full | LDS insts | VALU insts | MFMA insts |",
        "|---|---|---|---|---|---|---|---|",
    ]
    for f in order:
        a = p2.get(f)
        if not a or not a["SQ_BUSY_CYCLES"]:
            continue
        b = a["SQ_BUSY_CYCLES"]
        lines.append(f"| {f} | {a['SQ_LDS_IDX_ACTIVE'] / b:.3f} | {a['SQ_LDS_BANK_CONFLICT'] / b:.3f} | "
                     f"{a['SQ_LDS_DATA_FIFO_FULL'] / b:.3f} | {a['SQ_LDS_CMD_FIFO_FULL'] / b:.3f} | "
                     f"{a['SQ_INSTS_LDS']:.3e} | {a['SQ_INSTS_VALU']:.3e} | {a['SQ_INSTS_MFMA']:.3e} |")
    with open(os.path.join(ROOT, "profiles", "stalls_C2.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if len(sys.argv) != 2:
        sys.exit("usage: python profile_stalls.py OUT  (the directory the two rocprofv3 runs wrote into)")
    main(sys.argv[1])
