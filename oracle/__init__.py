"""CPU oracle for the IP-GFCCSD linear-solve path (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from this package.  The GPU library never
calls it and shares no code with it; both sides only share the seeded input
generator in ``synth``.

* ``oracle.fockspace`` -- O1: a Fock-space brute force.  It needs no working
  equations: it builds the second-quantised Hamiltonian, the cluster and
  de-excitation operators as determinant matrices and forms the connected
  similarity-transformed Hamiltonian, the ket ``abar_p|Phi>`` and the bra
  ``<Phi|(1+Lambda) abar_q^dagger`` directly from their definitions (paper,
  Theory section, eqs. for G_pq in the bi-orthogonal CC form and its compact form).
* ``oracle.ipgfcc`` -- O2: a matrix-free spin-adapted closed-shell
  implementation (intermediates, sigma product, diagonal, left vectors,
  GMRES, Green's function), pinned against O1 and closed forms.
* ``oracle.eagfcc`` -- O2 for the advanced (electron-attached) term: the
  spin-adapted 1p + 2p1h sigma product, its intermediates, diagonal, right-hand
  sides and left vectors, pinned against the N+1-sector brute force of O1.
* ``oracle.openshell`` -- the open-shell (spin-unrestricted) IP term: a brute
  force over both ionised sectors and the spin-orbital working equations,
  pinned against it and, for identical spins, against ``oracle.ipgfcc``.
"""
