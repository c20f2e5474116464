"""Parity bars shared by the GPU tests.

When only the summation order changes (rows and columns renumbered), the
oracle moves away from itself by its "spread"; the GPU sums in an order of
its own, so its distance from the oracle is another draw of the same kind.
The bar is SPREAD_FACTOR times the largest spread over the renumbered
copies, and never less than the absolute floor (1e-10 for iterates).
"""
SPREAD_FACTOR = 10


def bar(spread: float, floor: float = 1e-10) -> float:
    return max(floor, SPREAD_FACTOR * spread)


def ratio(err: float, spread: float) -> str:
    """err / spread, for the logs (inf when the oracle has no spread)."""
    return f"{err / spread:.1f}" if spread > 0 else ("0" if err == 0 else "inf")
