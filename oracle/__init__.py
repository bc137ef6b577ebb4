"""Plain FP64 CPU oracle for the GOCP ADAPT-VQE hot path.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import or run it.  The product path (the
HIP library and its Python binding) never calls into it, and it imports nothing
from the product.

Every function follows the paper's definitions (Eq. 1-6, Algorithm 1) as
directly as possible, in float64 / complex128, with no blocking, fusion or
reordering beyond what those definitions state.  Points where the paper is
silent or garbled take the readings listed in each module's docstring.

Modules
-------
pauli    -- Pauli strings and sums (Eq. 3), dense matrices for small registers
mapping  -- second-quantised Hamiltonian (Eq. 2) and JW / BK ladder operators
pool     -- spin-conserving singles + doubles pool (Sec. II.B, Table II)
gocp     -- non-commutativity graph and Largest-First colouring (Algorithm 1)
statevec -- energy (Eq. 1), gradients (Eq. 4), O(5) Taylor chain (Eq. 5-6)
adapt    -- the ADAPT growth loop with the line search reading
"""
