"""Kernel-class names the rocprofv3 summaries use, from mangled and demangled
kernel symbols.  Dense classes must be the names the library's own event
profiler reports (gcp_profile_read), or the traffic record and the bench
roofline would not line up; conv classes add the launch shape
(.w<waves>x<column tiles>), which the library's names leave out."""
import pytest

from paper_2208_05740_amd.profiling import class_of

CASES = [
    ("_ZN3gcp15gemm_epi_kernelIDF16bLi16ELi64ELi1ELi4ELi128ELb0ENS_6AdjEpiIDF16bLb0EEEEEvNS_8GemmArgsET6_",
     "adj.bf16.t16x64"),
    ("_ZN3gcp15gemm_epi_kernelIDF16bLi16ELi64ELi1ELi4ELi128ELb1ENS_6AdjEpiIDF16bLb0EEEEEvNS_8GemmArgsET6_",
     "adj.bf16.sign.t16x64"),
    ("_ZN3gcp15gemm_epi_kernelIDF16bLi16ELi64ELi1ELi4ELi128ELb1ENS_6AdjEpiIDF16bLb1EEEEEvNS_8GemmArgsET6_",
     "adj_pi.bf16.sign.t16x64"),
    ("_ZN3gcp15gemm_epi_kernelIDF16bLi32ELi32ELi2ELi2ELi128ELb0ENS_8BoundEpiIDF16bLb1EEEEEvNS_8GemmArgsET6_",
     "bound_pi.bf16.t32x32"),
    ("void gcp::gemm_epi_kernel<float, 32, 32, 2, 2, 64, false, gcp::BoundEpi<float, false> >",
     "bound.fp32.t32x32"),
    ("void gcp::gemm_epi_kernel<float, 32, 32, 2, 2, 64, false, gcp::BoundEpi<float, true> >",
     "bound_pi.fp32.t32x32"),
    ("_ZN3gcp15gemm_epi_kernelIDF16bLi64ELi64ELi2ELi2ELi128ELb0ENS_7ConcEpiEEEvNS_8GemmArgsET6_",
     "conc.bf16.t64x64"),
    ("_ZN3gcp16conv_slab_kernelIDF16bLi8ELi1ELb0ELb1ENS_6AdjEpiIDF16bLb0EEEEEvNS_8ConvArgsENS_8ConvPlanET4_",
     "conv_adj.bf16.sign.w8x1"),
    ("_ZN3gcp16conv_slab_kernelIDF16bLi8ELi1ELb0ELb0ENS_6AdjEpiIDF16bLb1EEEEEvNS_8ConvArgsENS_8ConvPlanET4_",
     "conv_adj_pi.bf16.w8x1"),
    ("void gcp::conv_slab_kernel<float, 8, 1, true, false, gcp::BoundEpi<float, true> >",
     "convT_bound_pi.fp32.w8x1"),
    ("_ZN3gcp16conv_slab_kernelIDF16bLi8ELi1ELb1ELb0ENS_7AhatEpiIDF16bEEEEvNS_8ConvArgsENS_8ConvPlanET4_",
     "convT_ahat.bf16.w8x1"),
    ("_ZN3gcp19convT_direct_kernelIfLi3ELi2ELi2ELi2ENS_7ConcEpiEEEvNS_8ConvArgsENS_8ConvPlanET4_",
     "convT_conc.fp32.direct.c3k2x2"),
    ("void gcp::convT_direct_kernel<__bf16, 1, 3, 3, 1, gcp::ConcEpi>", "convT_conc.bf16.direct.c1k3x3"),
    ("gcp::gamma_kernel", None),
    ("__amd_rocclr_copyBuffer", None),
]


@pytest.mark.parametrize("symbol,name", CASES)
def test_kernel_class_names(symbol, name):
    assert class_of(symbol) == name
