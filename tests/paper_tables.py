"""Readers for the values the paper prints, stored under tests/golden/."""
import os

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def error_table():
    """Table "error" (Section 5.4.1) as (sizes, [(lo, hi, [mape% per size])])."""
    sizes, rows = None, []
    with open(os.path.join(GOLDEN, "table_error_mape.txt")) as f:
        for line in f:
            line = line.strip()
            if line.startswith("# lo hi |"):
                sizes = [int(s) for s in line.split("|")[1].split()]
            elif line and not line.startswith("#"):
                rng, vals = line.split("|")
                lo, hi = (int(s) for s in rng.split())
                rows.append((lo, hi, [float(v) for v in vals.split()]))
    assert sizes is not None and all(len(r[2]) == len(sizes) for r in rows)
    return sizes, rows
