"""MI355X (gfx950) implementation of the Elfpie full-batch iteration (arXiv 2209.14671).

The computation lives in the HIP library built from ``csrc/`` (see ``build.py``);
``elfpie`` is the torch-facing binding of its C ABI (``include/elfpie.h``).
"""
from .elfpie import (F32, F32_MFMA_BF16X3, F64, FID_AMPLITUDE, FID_GAMMA, FID_INTENSITY, FID_LOG, LEARN_PUPIL, NORM_ANISO, NORM_ISO,  # noqa: F401
                     OPT_ADABELIEF, OPT_ELFPIE, OPT_NADAM, OPT_SGD, PUPIL_FILTER, PUPIL_SUPPORT, Batch, ElfpieError, ElfpieLoss, Plan, Problem, SpectrumFromObject,
                     State, elfpie_loss, elfpie_loss_object, grad_noalloc, problem_from_optics, workspace_bytes)
