"""CPU oracle for the block-sparse multiply and contraction.

TEST INFRASTRUCTURE ONLY.  Plain, slow numpy code in float64 that states
what the GPU library must compute.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product
package never does, and this package imports nothing from the product.  The
two share no code: only the seeded input generators in ``workloads`` feed
both.

Modules
-------
* ``blocksparse`` -- blocked matrices (Sec. 2: blocked CSR storage), block
  norms, the filtered set of block products, the multiply C = beta*C + alpha*A.B
  (Sec. 2: pairwise products of small dense blocks; Sec. 3: C = C + A x B),
  transposition, the stack (product list) and the gradient of the multiply.
* ``tensor`` -- block-sparse tensors and their contraction, directly and via
  the matrix mapping of Sec. 4.
* ``split`` -- emulation of the split-precision (bf16 pieces) product.

Parity status per function is stated in each module header.
"""
