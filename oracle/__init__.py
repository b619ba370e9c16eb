"""Oracle: plain CPU reference for tensor-network contraction.

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library or its binding.  It
shares no code with the GPU path.

  oracle.c / contract.py -- complex128 loop-nest contraction along a given
                            tree, with slicing and reverse mode
  statevector.py         -- brute-force statevector amplitudes (<= ~20 qubits)
  bruteforce.py          -- direct sum over all index values of the product of
                            leaf entries (tiny networks)
"""
