"""Writes profiles/traffic_pair_forces_n51200.json (read by bench.py) from
two rocprofv3 counter runs per kernel setting (FETCH_SIZE, then WRITE_SIZE,
each with a 256 MiB device-to-device copy first as the known-size
calibration kernel).

Usage: python bench_traffic.py OUT_DIR_PREFIX
where OUT_DIR_PREFIX_{FETCH_SIZE,WRITE_SIZE}_<v>_<s>_<f>_<cf>/pmc_counter_collection.csv
are the counter files of `bench.py --headline-only --tuning v,s,f,cf
--copy-calibration-mib 256`.  The sources hash ties the record to the
kernel sources it was measured on (bench.py ignores a stale record)."""
import collections
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["paper_1412_8502_amd/csrc/forces.hip", "paper_1412_8502_amd/csrc/fp64math.hpp",
           "paper_1412_8502_amd/csrc/internal.hpp", "paper_1412_8502_amd/csrc/list_items.hpp",
           "paper_1412_8502_amd/csrc/pair_items.hpp"]
SETTINGS = [(3, 32, 1, 0), (3, 0, 1, 1), (3, 0, 1, 2), (1, 0, 1, 1), (1, 0, 1, 2)]
# public coulomb_form -> the fused kernel's Coulomb template argument
FUSED_COULOMB_ARG = {0: 0, 1: 1, 2: 3}
COPY_KIB = 256 * 1024


def counters(path):
    acc = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        acc[(r["Kernel_Name"], r["Grid_Size"])].append(float(r["Counter_Value"]))
    return acc


def main(prefix):
    h = hashlib.sha256()
    for src in SOURCES:
        h.update(src.encode())
        h.update(open(os.path.join(ROOT, src), "rb").read())
    entries = []
    for t in SETTINGS:
        tag = "_".join(map(str, t))
        cf = FUSED_COULOMB_ARG[t[3]]
        kname = "k_forces_fused<MixedPolicy, 0, %d, %d>" % (t[0], cf)
        vals, factors = {}, {}
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            acc = counters("%s_%s_%s/pmc_counter_collection.csv" % (prefix, c, tag))
            copy = [v for (n, g), vs in acc.items() if "copyBuffer" in n and g == "131072"
                    for v in vs]
            kern = [v for (n, g), vs in acc.items()
                    if "k_forces_fused<pasta::MixedPolicy, 0, %d, %d>" % (t[0], cf) in n
                    for v in vs]
            factors[c] = COPY_KIB / (sum(copy) / len(copy))
            vals[c] = (sum(kern) / len(kern), len(kern), sum(copy) / len(copy))
        b = (vals["FETCH_SIZE"][0] * factors["FETCH_SIZE"] +
             vals["WRITE_SIZE"][0] * factors["WRITE_SIZE"]) * 1024
        entries.append({"kernel": kname, "tuning": list(t),
                        "fetch_kib": round(vals["FETCH_SIZE"][0], 1),
                        "write_kib": round(vals["WRITE_SIZE"][0], 1),
                        "dispatches": vals["FETCH_SIZE"][1],
                        "fetch_factor": round(factors["FETCH_SIZE"], 4),
                        "write_factor": round(factors["WRITE_SIZE"], 4),
                        "copy_fetch_kib": round(vals["FETCH_SIZE"][2], 1),
                        "copy_write_kib": round(vals["WRITE_SIZE"][2], 1),
                        "bytes_per_launch": int(round(b))})
    rec = {"workload": "n51200_yp020_n0.080", "sources": SOURCES,
           "sources_sha256": h.hexdigest(),
           "calibration": "256 MiB device-to-device copy (__amd_rocclr_copyBuffer, grid 131072)",
           "summary": "profiles/pair_forces_n51200.md", "entries": entries}
    with open(os.path.join(ROOT, "profiles", "traffic_pair_forces_n51200.json"), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main(sys.argv[1])
