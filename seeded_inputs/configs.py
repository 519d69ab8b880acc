"""The concrete synthetic workloads as JSON: one file per workload under
configs/ at the repository root, written from the generator definitions in
this package (python -m seeded_inputs.configs). The files record what the
tests and bench.py draw: sizes, primes (decimal strings, exact), seeds and
the generator parameters; tests/test_inputs.py checks that they still match."""
from __future__ import annotations

import json
import os

from . import (BASE_SEED, batched_jobs, batched_primes, serving_primes, workload_ct_n14, workload_polymul_n16,
               workload_single_u32)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CONFIG_DIR = os.path.join(ROOT, "configs")

GENERATOR = ("SplitMix64 stream per seed; a residue mod q is the next output shifted right by "
             "64 - bitlen(q), redrawn while >= q, drawn in memory order [poly][limb][coef]")


def _plain(w, role):
    return {"workload": w.name, "role": role, "N": w.N, "limbs": len(w.moduli), "polys": w.batch,
            "word_bits": w.word, "moduli": [str(q) for q in w.moduli], "seed": w.seed, "note": w.note,
            "generator": GENERATOR}


def workload_configs() -> dict[str, dict]:
    """Every workload, keyed by its name."""
    out = {}
    for w, role in ((workload_single_u32(), "parity and single-call latency"),
                    (workload_ct_n14(), "parity and single-call latency"),
                    (workload_polymul_n16(), "headline: forward + product + inverse of 2 ciphertexts")):
        out[w.name] = _plain(w, role)
    jobs = batched_jobs()
    out["batched_uneven_256polys"] = {
        "workload": "batched_uneven_256polys", "role": "batched executor (one graph launch)",
        "polys": len(jobs), "seed": BASE_SEED + 3, "word_bits": 64,
        "rule": "N uniform on {2^12..2^16}, L uniform on 1..32; polynomial i uses the first L primes",
        "primes": [str(q) for q in batched_primes()],
        "jobs": [{"N": j.N, "L": j.L} for j in jobs],
        "ntts": sum(j.L for j in jobs), "coefficients": sum(j.L * j.N for j in jobs),
        "generator": GENERATOR}
    out["serving_poisson_ntt_polymul"] = {
        "workload": "serving_poisson_ntt_polymul", "role": "serving loop (continuous batching)",
        "seed": BASE_SEED + 4, "word_bits": 64,
        "rule": ("Poisson arrivals (exponential gaps at the offered rate); 50% forward-NTT, 50% poly-mult jobs; "
                 "N uniform on {2^12..2^17}, L uniform on 1..40; a job uses the first L primes"),
        "primes": [str(q) for q in serving_primes()],
        "warmup_jobs": 1000, "measured_jobs": 20000, "offered_jobs_per_s": 15000.0,
        "load_curve_fractions_of_burst_rate": [0.3, 0.5, 0.7], "hbm_budgets_GiB": [0.5, 1, 4, 16],
        "generator": GENERATOR}
    return out


def write(directory: str = CONFIG_DIR) -> list[str]:
    os.makedirs(directory, exist_ok=True)
    paths = []
    for name, cfg in workload_configs().items():
        p = os.path.join(directory, name + ".json")
        with open(p, "w") as fh:
            json.dump(cfg, fh, indent=1)
            fh.write("\n")
        paths.append(p)
    return paths


if __name__ == "__main__":
    for p in write():
        print(p)
