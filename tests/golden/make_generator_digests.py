"""Write generator_sha256.json: SHA-256 of the float32 fields per seed.

Calls only the seeded input generator (no solver).  Re-run it only when the
generator is changed on purpose, and say why in the commit message.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_2301_12010_amd import inputs  # noqa: E402

CASES = {
    "dam_break": lambda: inputs.dam_break(),
    "parabolic_bowl": lambda: inputs.parabolic_bowl(),
    "steady_slope": lambda: inputs.steady_slope(perturb=0.05),
    "lake_at_rest": lambda: inputs.lake_at_rest(),
    "random_wet_33x17_s9": lambda: inputs.random_wet(33, 17, seed=9, dry_fraction=0.05),
    "large_coast_256_s2": lambda: inputs.large_coast(256, 256, 5.0, seed=2),
    "mitigation_256_s1000": lambda: inputs.mitigation_coast(256, 256, 2.0, seed=1000),
    "mitigation_1024_s1003": lambda: inputs.mitigation_coast(1024, 1024, 2.0, seed=1003),
    "uneven_s7": lambda: inputs.uneven_scenario(7),
    "deep_ocean_s5": lambda: inputs.deep_ocean(),
    "still_coast_s11": lambda: inputs.still_coast(),
}


def digests():
    return {k: f().digest() for k, f in CASES.items()}


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "generator_sha256.json")
    d = digests()
    d["uneven_plan_first8"] = [[list(s), n] for s, n in inputs.uneven_plan()[:8]]
    with open(out, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    print(out)
