"""Record comparison for tests: two records are the same when every field
is equal, NaN fields matching NaN (the undefined jackknife fields)."""
import math


def same_record(a: dict, b: dict) -> bool:
    if a.keys() != b.keys():
        return False
    for k in a:
        x, y = a[k], b[k]
        if isinstance(x, float) and isinstance(y, float) and math.isnan(x) and math.isnan(y):
            continue
        if x != y:
            return False
    return True
