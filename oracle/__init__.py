"""CPU oracle for the adaptive partitioned-index search (test infrastructure).

This package is test infrastructure, not part of the product: only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it.
It is a plain, slow, FP64 NumPy restatement of what the search computes:

* ``knn``     exact k-NN and recall@k (problem statement, Sec. 2.1)
* ``ivf``     fixed-nprobe partition scan and the nearest-centroid
              assignment invariant (Sec. 3, index structure)
* ``aps``     the spherical-cap recall model and Adaptive Partition
              Scanning (Sec. 5, Eqs. aps-pi / aps-p0 / aps-pi-final,
              Algorithm "Adaptive Partition Scanning")
* ``twolevel`` search through a two-level index (Sec. 3 and Sec. 5; the
              upper level's recall target is fixed, Sec. 5.1 / Table
              two_level_results)
* ``updates`` batched insert / delete replay (Sec. 2.1 and Sec. 3)
* ``kmeans``  Lloyd iterations used only to check the device build's
              objective (Sec. 3; parity unpinned for the centroids)
* ``maintenance`` the cost model, split / delete deltas, the estimate ->
              verify -> commit workflow and the split, refinement and delete
              actions on vectors (Sec. 4, Eqs. CostPartition, CostTotal,
              DeltaC, delta_split_exact, delta_merge_exact, delta_split_est)
* ``pq``      product-quantized rows and the scan over their codes with an
              exact rerank (Sec. 8, "Vector Compression")

It shares no code, headers, tables or constants with the device path.
"""
