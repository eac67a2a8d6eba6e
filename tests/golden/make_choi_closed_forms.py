"""Evaluates the paper's printed closed forms for the Choi-state entanglement of formation
(appendix on optimal Kraus decompositions for the Choi state).  Writes
choi_closed_forms.txt next to this file.  Uses only the formulas, no oracle code."""
import math
import os


def h(x):
    return -sum(t * math.log2(t) for t in (x, 1 - x) if t > 0)


rows = []
for p in (0.005, 0.01, 0.02, 0.1, 0.3):
    rows.append(("dephasing", p, h((1 + math.sqrt((2 - p) * p)) / 2)))
for g in (0.005, 0.01, 0.1, 0.3, 0.7):
    rows.append(("amplitude_damping", g, h((1 + math.sqrt(g)) / 2)))
for p in (0.005, 0.01, 0.02, 0.1, 0.3, 0.6):
    rows.append(("depolarizing", p, h((2 + math.sqrt(3) * math.sqrt((4 - 3 * p) * p)) / 4)))
out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "choi_closed_forms.txt")
with open(out, "w") as f:
    f.write("# channel rate EoF(Choi state) -- closed forms of the appendix on optimal Kraus\n")
    f.write("# decompositions for the Choi state (dephasing, amplitude damping, depolarizing)\n")
    for name, r, e in rows:
        f.write(f"{name} {r!r} {e!r}\n")
