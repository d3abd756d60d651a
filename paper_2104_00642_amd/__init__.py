"""MI355X-native hot path of the YUNIC particle-in-cell method (arXiv:2104.00642).

The computation lives in ``libpic.so`` (HIP kernels for gfx950 behind the C ABI
of ``include/pic.h``); ``_lib`` marshals arguments, ``sim`` sequences the calls
of one step, ``workloads`` makes seeded synthetic inputs.
"""
from ._lib import (PIC_BC_PERIODIC, PIC_F_CAPACITY, PIC_F_NONFINITE, PIC_F_OFFSET,  # noqa: F401
                   PIC_F_STRAGGLER, PIC_FP32_MIXED, PIC_FP64_PLAIN, PIC_QED_MLP, PIC_QED_TABLE, Config,
                   Context, Fields, Particles, PicError, Species, pic_check, pic_destroy,
                   pic_gather_push_deposit, pic_get_layout, pic_init, pic_last_error, pic_mlp_forward,
                   pic_mlp_grad, pic_mlp_train, pic_qed_step, pic_qed_table_lookup,
                   pic_qed_training_data, pic_sort, pic_yee_step)
