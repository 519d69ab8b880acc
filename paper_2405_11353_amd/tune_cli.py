"""Build the tuning table shipped next to libntt.so.

Runs ntt_autotune on the current GPU for every (word size, N, batch size) in a
grid covering the library's workloads and writes tune_<arch>.json into the
package directory, where the library loads it by default. Usage (on the GPU):

    python -m paper_2405_11353_amd.tune_cli [--quick]
"""
from __future__ import annotations

import argparse
import json
import os

from . import ntt as _ntt

PKG = os.path.dirname(os.path.abspath(__file__))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="fewer sizes and repetitions")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    import torch

    assert torch.cuda.is_available()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    out = args.out or os.path.join(PKG, f"tune_{arch}.json")
    # start from an empty table (not the shipped one)
    _ntt.ntt_tune_clear()
    reps = 5 if args.quick else 20
    grid = []
    for logn in range(4, 18):
        for items in (1, 8, 48, 96, 384, 1536):
            if (1 << logn) * items > (1 << 28):
                continue
            grid.append((64, logn, items))
    for logn in (10, 12, 14, 16):
        for items in (1, 64, 1024):
            grid.append((32, logn, items))
    if args.quick:
        grid = [g for g in grid if g[2] in (1, 96, 1536) or g[0] == 32]
    results = []
    for word, logn, items in grid:
        c = _ntt.ntt_autotune(1 << logn, items=items, reps=reps, flags=_ntt.NTT_WORD32 if word == 32 else 0)
        results.append({"word": word, "log_n": logn, "items": items, **c})
        print(json.dumps(results[-1]), flush=True)
    _ntt.ntt_tune_save(out)
    print(f"wrote {out}")


if __name__ == "__main__":
    main()
