"""Command-line runner: one simulation through libkk, its observables as a time
series (Results, "Cluster Analysis": average cluster size over time; the
fraction of similar first neighbours of "Image analysis"), one JSON object
per line.

    python -m paper_1309_4349_amd.run --geometry triangular --L 404 --x 0.3 \\
        --omega 0.9 --sweeps 100000 --every 1000 --start segregated

Every record holds the sweep counter, N_AB, E/kT, the exact and the
random-neighbour similar fractions, the number of clusters of --species and
their number- and weight-average and largest sizes.  --hist-out writes the
final cluster-size histogram (size, count) as JSON and --lattice-out the
final lattice (numpy .npy, one byte per site); --resume continues from a
lattice written by --lattice-out together with its sweep counter.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import kk


def parse(argv=None) -> argparse.Namespace:
    ap = argparse.ArgumentParser(prog="python -m paper_1309_4349_amd.run", description=__doc__.split("\n\n")[0])
    ap.add_argument("--geometry", choices=("square", "triangular"), default="triangular")
    ap.add_argument("--scheme", choices=("classes", "mpkk"), default="classes",
                    help="triangular only: the conflict-free classes or the paper's literal MPKK")
    ap.add_argument("--L", type=int, default=404, help="sites per row")
    ap.add_argument("--rows", type=int, default=0, help="triangular only: rows (0 = L)")
    ap.add_argument("--x", type=float, default=0.5, help="composition: fraction of type 1")
    ap.add_argument("--omega", type=float, default=0.9, help="omega / kT")
    ap.add_argument("--seed", type=int, default=0x13094349)
    ap.add_argument("--layout", choices=("auto", "int8", "bitpacked"), default="auto", help="square only")
    ap.add_argument("--start", choices=("random", "segregated"), default="random")
    ap.add_argument("--sweeps", type=int, default=10000)
    ap.add_argument("--every", type=int, default=1000, help="sweeps between records")
    ap.add_argument("--species", type=int, choices=(0, 1), default=1)
    ap.add_argument("--hist-out", default="", help="write the final cluster histogram here (JSON)")
    ap.add_argument("--lattice-out", default="", help="write the final lattice here (.npy)")
    ap.add_argument("--resume", default="", help="continue from this .npy lattice ...")
    ap.add_argument("--resume-sweep", type=int, default=0, help="... whose sweep counter is this")
    a = ap.parse_args(argv)
    if a.every < 1 or a.sweeps < 0:
        ap.error("--every must be >= 1 and --sweeps >= 0")
    return a


def run(a: argparse.Namespace, out=sys.stdout) -> list:
    if a.geometry == "square":
        sim = kk.Sim(a.L, a.x, a.omega, a.seed, layout=a.layout)
    else:
        sim = kk.Sim(a.L, a.x, a.omega, a.seed, geometry="triangular", rows=a.rows or None, scheme=a.scheme)
    records = []
    with sim:
        if a.resume:
            sim.set_lattice(np.load(a.resume, allow_pickle=False), a.resume_sweep)
        elif a.start != "random":
            sim.restart(a.start)
        t0 = time.perf_counter()
        done = 0
        while done < a.sweeps:
            n = min(a.every, a.sweeps - done)
            sim.sweep(n)
            done += n
            rec = sim.observe(a.species)
            rec["wall_s"] = time.perf_counter() - t0
            records.append(rec)
            out.write(json.dumps(rec) + "\n")
            out.flush()
        if a.hist_out:
            with open(a.hist_out, "w") as f:
                json.dump(sim.cluster_hist(a.species), f)
        if a.lattice_out:
            np.save(a.lattice_out, sim.get_lattice(), allow_pickle=False)
    return records


def main(argv=None) -> int:
    run(parse(argv))
    return 0


if __name__ == "__main__":
    sys.exit(main())
