"""FP64 CPU oracle for AdANNS-IVF / IVF-(O)PQ search.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, obviously correct
reference that the GPU library is checked against. Only the test suite, the
smoke entry point and the CPU-baseline leg of the benchmark may import it; the
library itself never does, and shares no code, constants or helpers with it.
Inputs come from the ``synth`` generator (random numbers only) or from the
caller; every floating-point step runs in float64 unless a function says that
the paper's method fixes another precision (the quantisers of the precision
form, which reproduce a storage format exactly).

Modules and the passages they follow:

* ``exact``     exact k-NN (brute force), Section 2 and Appendix C (k-Recall@N
                ground truth)
* ``kmeans``    Lloyd's k-means and the inverted lists, Section 3 ("Inverted
                File Index"), Algorithm 1 (construction)
* ``ivf``       AdANNS-IVF search, Algorithm 1 (inference) and the retrieval
                formulas of Table "formula" (Appendix A)
* ``pq``        PQ / OPQ training, encoding and ADC search, Section 3
                ("Optimized Product Quantization"), Section 4.2, Section 4.3
* ``precision`` BF16 / FP8-e4m3 storage formats and the shortlist-then-rerank
                form, Section 4.3 (shortlist, then rerank with a high-d MR)
* ``metrics``   k-Recall@N, the compute cost model (Appendix B.1), relative
                contrast (Appendix H.2), centroid recall (Appendix E.2)
* ``check``     tie-aware comparison of a candidate result with the oracle

Parity status of each function is stated in its module header.
"""
from . import exact, kmeans, ivf, pq, precision, metrics, check  # noqa: F401
