"""Writes tests/data/manifest.json: the SHA-256 of every generated workload
(alphabet, offsets and residue codes, as SeqSet.sha256 hashes them) and of its
homology ids, so that a change of the generator or its RNG cannot silently
change the inputs that stand in for the paper's data sets.

Run from the repository root: python tests/data/make_manifest.py
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from workloads import CONFIGS, make_inputs  # noqa: E402


def digests(s):
    h = hashlib.sha256(np.ascontiguousarray(s.homology, dtype=np.int64).tobytes()).hexdigest()
    return {"n": s.n, "residues": int(s.offsets[-1]), "sha256": s.sha256(),
            "homology_sha256": h}


def main():
    out = {"generator": "workloads.generate (SplitMix64 streams per family, seed 0x09012742 + "
                        "workload index)",
           "workloads": {name: digests(make_inputs(name)) for name in CONFIGS}}
    with open(os.path.join(HERE, "manifest.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
