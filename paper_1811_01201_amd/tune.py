"""Measure the batched launch's team configurations on this device and
write the tuning table (JSON) that APSP_TUNE_TABLE points the library at.

    python -m paper_1811_01201_amd.tune --out apsp_tune.json
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default="apsp_tune.json")
    ap.add_argument("--graphs-per-class", type=int, default=0)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    import paper_1811_01201_amd as apsp

    report = {}
    for dtype in ("int32", "float32"):
        for pred in (False, True):
            r = apsp.batch_autotune(dtype, pred, args.graphs_per_class, args.reps)
            report[f"{dtype}/{'pred' if pred else 'dist'}"] = r
            print(dtype, "pred" if pred else "dist", json.dumps(r), flush=True)
    apsp.tune_save(args.out)
    print("wrote", args.out, flush=True)


if __name__ == "__main__":
    main()
