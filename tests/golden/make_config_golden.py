"""Writes tests/golden/config_results.json: the oracle's FindRepeats result on
the full-size synthetic configurations that the oracle is too slow to rerun
inside a GPU test (n = 2^24), with SHA-256 digests of its whole suffix array
and LCP array (little-endian uint32, the LCP array of length n-1) and its
per-round active suffix counts.  Calls only oracle/ and the input generators.

    python tests/golden/make_config_golden.py
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2406_18111_amd import synth  # noqa: E402


def main():
    out = {"_about": "Oracle (oracle/findrepeats_ref.c) results on full-size synthetic inputs; "
                     "regenerate with this script.", "configs": {}}
    for name, gen in (("config2_n2^24_u32", synth.config2),):
        t, m = gen()
        t0 = time.time()
        r = oracle.find_repeats(t, m, with_stats=True)
        sa, act = oracle.suffix_array(t, return_active=True)
        lcp = oracle.lcp(t, sa)
        sa_sha = hashlib.sha256(sa.astype("<u4").tobytes()).hexdigest()
        lcp_sha = hashlib.sha256(lcp.astype("<u4").tobytes()).hexdigest()
        del sa, lcp
        out["configs"][name] = {
            "min_len": m,
            "n": int(len(t)),
            "occurrences": [[int(a), int(b)] for a, b in zip(r["occ_start"], r["occ_len"])],
            "rows": [[int(a), int(b), int(c)] for a, b, c in zip(r["row_start"], r["row_len"], r["row_count"])],
            "stats": r["stats"],
            "sa_sha256": sa_sha,
            "lcp_sha256": lcp_sha,
            "active_per_round": [int(a) for a in act],
            "oracle_seconds": round(time.time() - t0, 1),
        }
        print(name, out["configs"][name]["stats"], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "config_results.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
