"""Plain FP64 CPU oracle of Fuzzy C-Means on grey levels.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
anything in this package: only ``tests/``, the smoke check and the CPU-baseline
leg of the benchmark may.  It shares no code with the HIP library (different
files, different formula form, different precision) and is pinned against
what the paper and mathematics fix (see ``tests/test_oracle_pins.py``).

Modules
  fcm_ref    literal Eq.1-Eq.4 / Algorithm 1 per voxel (numpy, FP64)
  fcm_hist   the same sums regrouped over the 256 grey levels (exact regrouping)
  fcm_fast   the per-voxel iteration in plain C, threaded over the host cores
             (fcm_fast.c; for timing and large sizes)
  exact      the same iteration in exact rational (m = 2, 3) or 60-digit
             decimal arithmetic, for tiny inputs
  mlp_ref    FP64 forward/backward of the histogram -> centroid network
  dice       confusion counts and the Dice coefficient of Eq.5 per tissue
"""
