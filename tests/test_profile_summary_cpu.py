"""Kernel-name classification of the rocprofv3 summaries: every conjugation
kernel variant maps to the class the library's own profiler reports."""

from paper_2604_15765_amd import profile_summary as ps


def test_kernel_class():
    cases = {
        "ht::conj_kernel<double, 1, 1, 0, 3>": "c128_k1_c1_direct",
        "ht::conj_kernel<float, 2, 0, 1, 0>": "c64_k2_c0_transfer",
        "ht::native_kernel<double, 1, 0, 3, 16, 0>": "c128_k1_c0_native",
        "ht::native_kernel<float, 3, 2, 0, 32, 1>": "c64_k3_c2_native",
        "ht::k3_kernel<double, 1, 3>": "c128_k3_c1_kraus",
        "ht::pair_kernel<1, 1, 0, 3, 2>": "c64_k1_c1_direct",
        "ht::pair_kernel<1, 0, 1, 0, 2>": "c64_k1_c0_transfer",
        "ht::pair_kernel<2, 2, 0, 3, 1>": "c64_k2_c2_direct",
        "ht::conj_sync_kernel<double, 1, 1, 1, 3>": "c128_k1_c1_transfer",
        "ht::conj_pipe_kernel<double, 2, 2, 0, 3, 512, true>": "c128_k2_c2_direct",
        "ht::stage_kernel<double, 1, 0, 512, true>": "c128_k1_c0_direct",
        "ht::stage_kernel<float, 2, 1, 256, false>": "c64_k2_c0_transfer",
        "ht::stage_kernel<double, 1, 1, 512, true, true>": "c128_k1_c0_transfer",
        "ht::pair_sync_kernel<1, 1, 1, 3, 2, 1024>": "c64_k1_c1_transfer",
        "ht::pair_sync_kernel<2, 2, 0, 0, 1, 512>": "c64_k2_c2_direct",
        "ht::pair_diag_kernel<2, 2, 0, 3>": "c64_k2_c2_direct_diag",
        "ht::stage_kernel<float, 2, 0, 512, false, true>": "c64_k2_c0_direct",
        "ht::trace_partial_kernel<double>": None,
        "ht::batch_kernel<float>": None,
    }
    for name, cls in cases.items():
        assert ps.kernel_class(name) == cls, name
