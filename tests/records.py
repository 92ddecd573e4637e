"""Error figures of the parity tests, printed at the end of the pytest run
(terminal summary), so that a quiet run (-q) still shows them."""

RECORDS = []


def record(*fields):
    RECORDS.append(" ".join(f"{f:.3e}" if isinstance(f, float) else str(f) for f in fields))
