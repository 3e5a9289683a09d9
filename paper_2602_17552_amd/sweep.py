"""Missed critical points: plain SZp against TopoSZp.

For stand-ins of the paper's five CESM datasets (their grid shapes, synthetic
values; see datagen.climate_stand_in) and the absolute bounds of its Table II
(1e-3, 1e-4, 1e-5), compresses every field with the plain SZp stream
(topo=0) and with TopoSZp, decompresses on the GPU, and counts false
negatives, positives and types with the library's GPU evaluator.  Reports
the averages per dataset and bound with the bit rate of each.

    python -m paper_2602_17552_amd.sweep --fields 3 --out sweep.md
"""
from __future__ import annotations

import argparse
import json
import sys


def run(fields_per_set: int = 3, bounds=(1e-3, 1e-4, 1e-5), sets=None):
    import numpy as np
    import torch

    import paper_2602_17552_amd as tsz
    from paper_2602_17552_amd import datagen

    sets = sets or list(datagen.CLIMATE_SHAPES)
    rows = []
    for name in sets:
        fields = [torch.from_numpy(datagen.climate_stand_in(name, seed=k)).cuda() for k in range(fields_per_set)]
        for eb in bounds:
            for mode in ("SZp", "TopoSZp"):
                acc = {"FN": 0, "FP": 0, "FT": 0, "cps": 0, "bits": 0.0, "max_err_over_e": 0.0, "failed": 0}
                for f in fields:
                    st, s = tsz.compress(f, eb, "abs", topo=(mode == "TopoSZp"))
                    if st != tsz.OK:
                        acc["failed"] += 1
                        continue
                    st, rec = tsz.decompress(s, tuple(f.shape))
                    if st != tsz.OK:
                        acc["failed"] += 1
                        continue
                    ev = tsz.eval_topology(f, rec)
                    acc["FN"] += ev["FN"]
                    acc["FP"] += ev["FP"]
                    acc["FT"] += ev["FT"]
                    acc["cps"] += ev["cp_min"] + ev["cp_sad"] + ev["cp_max"]
                    acc["bits"] += 8.0 * s.numel() / f.numel()
                    acc["max_err_over_e"] = max(acc["max_err_over_e"], ev["max_err"] / eb)
                k = max(1, len(fields) - acc["failed"])
                rows.append({"dataset": name, "shape": list(datagen.CLIMATE_SHAPES[name]), "eb": eb,
                             "compressor": mode, "fields": len(fields), "failed": acc["failed"],
                             "FN": acc["FN"] / k, "FP": acc["FP"] / k, "FT": acc["FT"] / k,
                             "critical_points": acc["cps"] / k, "bits_per_value": round(acc["bits"] / k, 3),
                             "max_err_over_eb": round(acc["max_err_over_e"], 4)})
                print(json.dumps(rows[-1]), flush=True)
    return rows


def markdown(rows, command: str) -> str:
    out = ["# Missed critical points: plain SZp vs TopoSZp (synthetic stand-ins)", "",
           "Command (repo root, one MI355X): `%s`" % command, "",
           "Averages per field. Fields: 64 plane waves + N(0, 1e-2^2) noise, normalised to [0, 1], "
           "on the grid shapes of the paper's CESM datasets; absolute bounds as in its Table II.", "",
           "| dataset | shape | bound | compressor | FN | FP | FT | critical points | bits/value | max err / bound |",
           "|---|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        out.append("| %s | %s | %g | %s | %.1f | %.1f | %.1f | %.0f | %.3f | %.3f |" % (
            r["dataset"], "x".join(map(str, r["shape"])), r["eb"], r["compressor"], r["FN"], r["FP"], r["FT"],
            r["critical_points"], r["bits_per_value"], r["max_err_over_eb"]))
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--fields", type=int, default=3, help="fields per dataset")
    ap.add_argument("--out", default=None, help="markdown table to write")
    ap.add_argument("--json", default=None, help="rows as JSON to write")
    args = ap.parse_args(argv)
    rows = run(args.fields)
    cmd = "python -m paper_2602_17552_amd.sweep " + " ".join(sys.argv[1:] if argv is None else argv)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(markdown(rows, cmd.strip()))
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(rows, fh, indent=1)


if __name__ == "__main__":
    main()
