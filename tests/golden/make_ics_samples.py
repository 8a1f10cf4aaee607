"""Writes ics_samples.json: a few generated bodies per workload, pinning the
generator's draw order and element conversion (the inputs, not any result of
the method).  Run from the repository root: python tests/golden/make_ics_samples.py"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import solar_ics as S  # noqa: E402

out = {"note": "first, middle and last body of each workload: pos[3], vel[3], mass"}
for key, sysd in [("0", S.config(0)), ("1", S.config(1)), ("2", S.config(2)),
                  ("3.0", S.config(3, 0)), ("3.511", S.config(3, 511)), ("4", S.config(4))]:
    idx = [1, sysd.n // 2, sysd.n - 1]
    out[key] = {"n": sysd.n, "counts": sysd.counts,
                "bodies": {str(i): {"pos": sysd.pos[:, i].tolist(), "vel": sysd.vel[:, i].tolist(),
                                    "mass": float(sysd.mass[i])} for i in idx}}
path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ics_samples.json")
with open(path, "w") as f:
    json.dump(out, f, indent=1)
print("wrote", path)
