"""FP64 CPU oracle for the smoothed BF16 GEMM stack -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  It shares no code with the GPU library (``paper_2605_29752_amd``) and
never imports it.  Parts:

* ``gemm``     -- plain FP64 GEMM and the |A||B| normaliser (C library ``liboracle.so``).
* ``dp``       -- the padding (T1) and split-plus-padding (T2) tables, literal recurrences.
* ``enumerate``-- exhaustive optimum over pad/split plan trees (pins ``dp``).
* ``metrics``  -- TFLOPs, mean, roughness, 3-D aggregate, ideal landscape, decomposition.
* ``memstudy`` -- statistics of the buffer read/write study (slowdown, rank correlation,
                 spread across N, warm-up drift).
"""
from .gemm import (build_oracle, lib, gemm_f64, gemm_entries, scaled_err, bf16_to_f64,
                   f64_to_bf16_rne)  # noqa: F401
