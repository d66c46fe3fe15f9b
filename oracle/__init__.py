"""CPU oracle for the uniform H-matrix matrix-vector product.

TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg
may import, call, link or execute anything under oracle/.  The product path (the HIP
library and its binding) never does, and the oracle imports nothing from the product
package: it reads an operator through the documented host layout (a mapping of plain
numpy arrays, see ``uniform.OPERATOR_KEYS``) and evaluates the kernel itself.

Modules
-------
kernel   the Helmholtz single-layer point kernel and brute-force dense products
uniform  the uniform H-matrix product by its definition, block by block (Definition 2.4),
         the H-matrix product by its definition (Definition 2.3), the optimal cluster
         basis of Algorithm 1, and bindings to the C implementations of Algorithms 5 and 6
aca      ACA with partial pivoting (section 2.3) and kernel blocks by position, for the
         construction kernels
build    compiles uhm_oracle.c into liboracle.so with gcc

Parity status: every function here is pinned by a ``-m "not gpu"`` test; see
tests/test_oracle_pins.py for which property pins which function.
"""
