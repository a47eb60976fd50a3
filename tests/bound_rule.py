"""The bound-based stopping rule of fftgal_set_bound_tol, applied to a
sequence of CG energies.

The library documents the rule (include/fftgal.h): after at least two steps,
stop once the last decrease d_k = energy_{k-1} - energy_k satisfies
d_k <= btol |energy_k| (1 - q) with q = d_k / d_{k-1} clipped to [0, 0.99]
(the remaining decrease, estimated as d_k q / (1 - q), is then below btol
times the entry).  It is a stopping heuristic of the library, not part of the
paper's method, so it is stated here, beside the tests that check it, and not
in the oracle: the oracle supplies the exact energy of every CG iterate
(Sec. 6.4), and these tests check the library's stopping iteration and the
quality of the bounds it returns against them.
"""


def first_stop(energies, btol):
    """First iteration k >= 2 at which the rule stops, or None."""
    for k in range(2, len(energies)):
        dk = energies[k - 1] - energies[k]
        dprev = energies[k - 2] - energies[k - 1]
        if dprev > 0.0:
            q = min(max(dk / dprev, 0.0), 0.99)
            if dk <= btol * abs(energies[k]) * (1.0 - q):
                return k
    return None
