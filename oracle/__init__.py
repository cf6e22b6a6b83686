"""CPU oracle: a plain, slow, complex128 reference of what the tensor-network
simulator computes.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The native library
never calls it, and it shares no code with the native library: gate
matrices, Kraus sets, the circuit-to-network mapping, the path cost model,
the greedy searches, the slicer, the MPS truncation and the learned scorer
are each written here independently, in numpy, from the paper's statement
of the method.

Modules
    gates       gate and Kraus matrices from their names
    statevector O1: brute-force state vector; amplitudes and marginal slices
    contract    O2: naive loop-nest pairwise contraction and whole-network
                contraction along a given pairwise path
    network     circuit -> tensor network (qubit wires become indices)
    paths       O6: path cost model, greedy / randomised greedy, slicing
    noise       O3 density matrix and O4 Kraus trajectories
    mps         O5: matrix-product-state simulator with SVD truncation
    gnn         O7: the contraction-order scorer, forward and backward, FP64
    observables Pauli-string expectation values: definition, conjugate
                (double-depth) network with light-cone collapse, and
                wave-function slicing

Parity pins are listed in each module header; functions without one say
"parity unpinned".
"""
