"""CPU oracle for Clifford-based circuit cutting (test infrastructure).

Plain, slow, obviously correct reference implementations of what the
circuit-cutting hot path computes, written from the paper (SuperSim,
Secs. III-B and V) and the works it cites for its building blocks
(Aaronson-Gottesman tableau simulation for the Clifford fragments, a dense
state vector for the non-Clifford fragments, the Pauli-basis wire-cutting
identity of Peng et al. for the recombination).

This package is test infrastructure.  Only the test suite, the smoke entry
point and the benchmark's CPU-baseline leg may import, link or run anything
in it; the product library never does, and it shares no code with it.
Floating point is fp64 throughout.

Modules
-------
philox        Philox4x32-10 counter-based generator (Salmon et al., SC'11).
statevector   brute-force dense state vector of the uncut circuit.
chp           literal Aaronson-Gottesman CHP tableau (plain C via ctypes).
stabilizer    GF(2) elimination on stabilizer generators: exact outcome
              distributions and Pauli expectations, independent of chp.
cutting       fragmenter, variants, fragment evaluation, Pauli transform,
              recombination, Z-string expectations.
mlp           fp64 MLP with hand-derived backprop and the importance
              estimator over cut terms.
"""
