"""Write the batched and served run sets (data/c4_runs.json,
data/c5_requests.json) from their seeded generators in workloads.py.

Usage: python -m paper_2404_10861_amd.make_workload_lists
"""
import json
import os

from . import workloads as wl


def main():
    os.makedirs(wl.DATA, exist_ok=True)
    with open(wl.C4_LIST, "w") as f:
        json.dump({"about": "batched workload: 64 runs [grid_w, grid_h, agents per island, "
                            "sites, kind, tournament, generations, seed], drawn by "
                            "workloads.c4()",
                   "runs": wl.c4_rows(wl.c4())}, f, separators=(",", ":"))
    with open(wl.C5_LIST, "w") as f:
        json.dump({"about": "served workload: Poisson arrivals at 20/s over 120 s [arrival s, "
                            "grid_w, grid_h, generations, kind, sites, seed]; 32 agents per "
                            "island, tournament of two, 1,024-agent query; drawn by "
                            "workloads.c5()",
                   "requests": wl.c5_rows(wl.c5())}, f, separators=(",", ":"))


if __name__ == "__main__":
    main()
