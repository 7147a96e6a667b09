"""Independent crystal-lattice enumeration for closed-form pins (integer lattice points only;
shares nothing with the oracle's pair search)."""
import itertools
import math
from collections import Counter


def fcc_shells(a, r_max):
    """Neighbour shells of an FCC lattice of cubic constant a: {distance: count} for 0 < r < r_max.
    FCC sites are the integer points (i, j, k) with i + j + k even, in units of a/2."""
    m = int(math.ceil(2.0 * r_max / a)) + 1
    shells = Counter()
    for i, j, k in itertools.product(range(-m, m + 1), repeat=3):
        if (i + j + k) % 2 or (i, j, k) == (0, 0, 0):
            continue
        n2 = i * i + j * j + k * k
        r = 0.5 * a * math.sqrt(n2)
        if r < r_max:
            shells[n2] += 1
    return {0.5 * a * math.sqrt(n2): c for n2, c in sorted(shells.items())}
