"""Writes geometry_hashes.json: sha256 of every workload's seeded solid mask.

Calls only the seeded input generators; it pins that the generators are
deterministic across machines and library versions.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2508_18202_amd import inputs  # noqa: E402


def table():
    ws = [inputs.small_block(), inputs.urban_les(), inputs.adjoint_case(), inputs.assimilation_case(), inputs.cylinder_gpc()] + inputs.uneven_cases()
    return {w.name: inputs.mask_hash(inputs.solid_mask(w)) for w in ws}


if __name__ == "__main__":
    with open(os.path.join(HERE, "geometry_hashes.json"), "w") as fh:
        json.dump(table(), fh, indent=1, sort_keys=True)
