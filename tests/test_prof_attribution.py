"""The profiler helper's attribution of kernel dispatches to the library's
timed regions (paper_2302_05002_amd/prof.py), which the traffic summaries
and `roofline.traffic` rest on: one 20M-point build as the trace lists it,
the same build with the binned quantise pass, with a two-pass chunk split
(found from the kernel names, or from a given number of passes) and with the
one-pass form.  Runtime copies belong to no region."""
from paper_2302_05002_amd import prof

# (region, kernel) of one build of the 20M-point planes workload, in launch order
BUILD = [
    ("preview", "k_preview_bits"), ("preview", "k_scan_small"), ("preview", "k_bits_write"),
    ("bbox", "k_bbox"), ("bbox", "k_setup"),
    ("quantize", "k_quantize<false, 1024, 14, 8>"),
    ("cut", "k_pyr_export"), ("cut", "k_pyr_level"), ("cut", "k_pyr_top"), ("cut", "k_cut_small"),
    ("cut", "k_cut_rank"), ("cut", "k_cut_index"), ("cut", "k_wc_chunks"), ("cut", "k_wc_segs"),
    ("chunk_split", "k_scan_small"), ("chunk_split", "k_u32_to_u64"), ("chunk_split", "k_scan_reduce"),
    ("chunk_split", "k_scan_down<true>"), ("chunk_split", "k_ms_count<false, 8>"),
    ("chunk_split", "k_scan_reduce"), ("chunk_split", "k_scan_down<true>"),
    ("chunk_split", "k_ms_scatter<false, 8, false>"),
    ("subsample", "k_ms_seg_prep_one"), ("subsample", "k_ms_count<true, 12>"), ("subsample", "k_scan_reduce"),
    ("subsample", "k_scan_top"), ("subsample", "k_scan_down<false>"), ("subsample", "k_ms_scatter<true, 12, false>"),
    ("subsample", "k_fill_many"), ("subsample", "k_list_classes"), ("subsample", "k_subsample_fast<64, 4, 10>"),
    ("subsample", "k_subsample_fast<512, 8, 13>"), ("subsample", "k_scan_reduce"), ("subsample", "k_scan_down<true>"),
    ("subsample", "k_decide"), ("subsample", "k_node_counts"), ("subsample", "k_scan_reduce"),
    ("subsample", "k_scan_down<true>"),
    ("node_counts", "k_np_pieces"), ("node_counts", "k_scan_reduce"), ("node_counts", "k_scan_down<true>"),
    ("node_counts", "k_np_shared"), ("node_counts", "k_np_count"),
    ("node_place", "k_fill_u32"), ("node_place", "k_node_fill"), ("node_place", "k_scan_small"),
    ("node_place", "k_np_lists"), ("node_place", "k_np_place"), ("node_place", "k_np_copy"),
    ("node_sort", "k_np_sort<64, 16, false, false>"), ("node_sort", "k_np_sort<512, 32, true, false>"),
    ("node_sort", "k_np_merge"), ("node_sort", "k_np_merge"), ("node_sort", "k_u32_to_u64"),
]


def _names(build):
    return [f"void fpo::{k}(WcArgs)" for _, k in build]


def _check(build, chunk_passes=0):
    got = prof.attribute(_names(build) * 2, chunk_passes)
    assert got == [r for r, _ in build] * 2


def test_table_form():
    _check(BUILD)


def test_runtime_copies_belong_to_no_region():
    names = _names(BUILD)
    names.insert(20, "__amd_rocclr_copyBuffer")
    got = prof.attribute(names)
    assert got[20] is None
    assert [r for r in got if r is not None] == [r for r, _ in BUILD]


def test_binned_quantise():
    i = BUILD.index(("quantize", "k_quantize<false, 1024, 14, 8>"))
    binned = BUILD[:i] + [("quantize", k) for k in ("k_qz_bin_code", "k_scan_reduce", "k_scan_down<true>",
                                                       "k_qz_bin_place", "k_qz_bin_grid")] + BUILD[i + 1:]
    _check(binned)


def test_two_pass_chunk_split():
    i = BUILD.index(("chunk_split", "k_ms_count<false, 8>"))
    second = [("chunk_split", "k_ms_count<false, 8>"), ("chunk_split", "k_scan_reduce"),
              ("chunk_split", "k_scan_down<true>"), ("chunk_split", "k_ms_scatter<false, 8, false>")]
    _check(BUILD[:i + 4] + second + BUILD[i + 4:], chunk_passes=2)
    _check(BUILD[:i + 4] + second + BUILD[i + 4:])   # found without the count


def test_one_pass_chunk_split():
    """The look-back form: a fill and one scatter, no counting pass."""
    i = BUILD.index(("chunk_split", "k_ms_count<false, 8>"))
    one = BUILD[:i - 4] + [("chunk_split", "k_scan_pair"), ("chunk_split", "k_fill_u32"),
                           ("chunk_split", "k_ms_scatter<false, 8, true>")] + BUILD[i + 4:]
    _check(one)
    _check(one, chunk_passes=1)
