"""Error bounds of the FP64 filter parity tests.

A filter pass of degree m applies M~^-1 once per degree step.  The
enrichment rows of each H^E apply come out of sums whose terms nearly cancel,
so their rounding is about eps (2^-53) of the terms, and M~^-1 magnifies it by
up to A (the 2-norm amplification of (M~^E)^-1, EFESystem.tilde_condition).
The recurrence carries every step's error forward with bounded growth, so the
errors add up over the m steps: relative error <= c m eps A.  c = 4 counts two
roundings per step (the apply's assembly and the recurrence update) and a
factor 2 for the growth of the scaled recurrence.  Short filters keep a floor
of 1e-14 A, the bound these tests used before the degree-dependent term."""
EPS = 2.0 ** -53


def filter_tol(degree, amplification, base=1e-11):
    return base + max(1e-14, 4.0 * degree * EPS) * amplification
