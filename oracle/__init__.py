"""Plain FP64 CPU oracle of the LDPC link: bits, encoder, Gray QAM mapper,
AWGN, demappers, belief-propagation decoders, weighted BP and its gradient,
neural demapper, error counting.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The GPU library never calls it and shares no code with it; the two
meet only in the seeded inputs of ``inputs/``.

The paper (Sionna white paper, arXiv 2203.11854) prints no equations.  What
it fixes is the order of the link (Sec. "Hello, World!", Listing 1), that
the channel and demapper take the noise variance, that LLRs are logits of
bit = 1 (Listing 2 feeds them to a binary cross-entropy with the code bits
as labels), batch-first tensors of independent Monte-Carlo trials (Sec.
"Design principles") and that the decoder family is belief propagation and
its variants such as min-sum (Sec. "Features" and "Custom CUDA kernels").
Every formula here is the textbook definition named in the docstring of the
function that computes it.

Conventions used throughout:

* Boundary LLR ``L = ln P(b=1)/P(b=0)``; the decoders work internally with
  ``lam = -L = ln P(b=0)/P(b=1)`` and decide ``b_hat = [APP < 0]``.
* Circulant ``P^s`` with ``s`` in ``[0, Z)``: check ``(i, r)`` joins variable
  node ``(j, (r + s) mod Z)``.
* Canonical edge order: decoded base nonzeros in row-major order
  ``e = 0..nnz-1``; edge id ``e * Z + r`` where ``r`` is the check's lift
  index.

Functions with no independent pin say "parity unpinned" in their docstring.
"""
