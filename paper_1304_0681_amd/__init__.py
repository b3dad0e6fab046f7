"""Python binding of libhpgsw (batched Smith-Waterman for RNA-seq reads on MI355X).

Argument marshalling only: every step of the alignment path runs in the HIP
kernels of ``libhpgsw.so``; PyTorch provides device memory and streams.  The
functions mirror the C ABI in ``include/hpgsw.h`` one to one.  If the library
is missing or no gfx950 device is present, the calls fail loudly; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhpgsw.so")

SW_OK, SW_E_INVALID, SW_E_RANGE, SW_E_NOMEM, SW_E_DEVICE, SW_E_NODEVICE, SW_E_STATE = \
    0, -1, -2, -3, -4, -5, -6
SW_WANT_ENDS = 1
SW_OPT_INT16 = 1
SW_OPT_BLOCKS_PER_CU = 2
SW_OPT_TB_SCRATCH_MB = 3
SW_NOALLOC_MAX_PAIRS = 1 << 22
# CIGAR op codes ((length << 4) | code)
SW_OP_M, SW_OP_I, SW_OP_D, SW_OP_N, SW_OP_S = 0, 1, 2, 3, 4
OP_NAMES = "MIDNS"

HIT_DTYPE = np.dtype([("score", "<i4"), ("read_end", "<i4"), ("ref_end", "<i4")])
ALN_DTYPE = np.dtype([("score", "<i4"), ("read_begin", "<i4"), ("read_end", "<i4"),
                      ("ref_begin", "<i4"), ("ref_end", "<i4"), ("n_ops", "<u4"),
                      ("status", "<u4")])
WINDOW_DTYPE = np.dtype([("read_id", "<u4"), ("ref_begin", "<u4"), ("len", "<u2"),
                         ("strand", "u1"), ("flags", "u1")])
CAL_DTYPE = np.dtype([("read_id", "<u4"), ("first", "<u4"), ("last", "<u4"), ("strand", "u1"),
                      ("valid", "u1"), ("reserved", "<u2")])
JUNCTION_DTYPE = np.dtype([("start", "<u8"), ("end", "<u8"), ("count", "<u4"),
                           ("strand", "<u4")])
REGION_DTYPE = np.dtype([("first", "<u4"), ("read_pos", "<u2"), ("strand", "u1"),
                         ("reserved", "u1")])
SW_SEEKER_MAX_CALS = 16
SW_SEEKER_MAX_REGIONS = 1024
SW_BMAP_MAX = 16
BMAP_DTYPE = np.dtype([("first", "<u4"), ("last", "<u4"), ("strand", "u1"), ("edits", "u1"),
                       ("op", "u1"), ("reserved", "u1"), ("edit_pos", "<i4")])


class SwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hpgsw status {status}: {msg}")
        self.status = status


class sw_scoring(ctypes.Structure):
    _fields_ = [("match", ctypes.c_int32), ("mismatch", ctypes.c_int32),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32)]


class sw_timing(ctypes.Structure):
    _fields_ = [("bucket_ms", ctypes.c_float), ("score_ms", ctypes.c_float),
                ("class_ms", ctypes.c_float * 16), ("class_path", ctypes.c_int32 * 16)]


class sw_batch(ctypes.Structure):
    _fields_ = [("d_ref2b", ctypes.c_void_p), ("ref_len", ctypes.c_uint64),
                ("d_reads2b", ctypes.c_void_p), ("reads_len", ctypes.c_uint64),
                ("d_read_off", ctypes.c_void_p), ("d_read_len", ctypes.c_void_p),
                ("n_reads", ctypes.c_uint32), ("d_win", ctypes.c_void_p),
                ("n_pairs", ctypes.c_uint32), ("d_n_pairs", ctypes.c_void_p)]


class sw_seed_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("step", ctypes.c_uint32), ("offset", ctypes.c_uint32),
                ("max_occ", ctypes.c_uint32)]


class sw_filter_params(ctypes.Structure):
    _fields_ = [("logit_lo", ctypes.c_float), ("logit_hi", ctypes.c_float),
                ("logit_drop", ctypes.c_float)]


SW_FEATURES = 64
SW_MLP_PARAMS = 24961


_lib = None


def lib() -> ctypes.CDLL:
    """Load libhpgsw.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_1304_0681_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, U32, U64, I32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
        L.sw_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(P)]
        L.sw_ctx_destroy.argtypes = [P]
        L.sw_last_error.argtypes = [P]
        L.sw_last_error.restype = ctypes.c_char_p
        L.sw_pack2b.argtypes = [P, P, U64, P, P, P]
        L.sw_batch_score.argtypes = [P, ctypes.POINTER(sw_batch), ctypes.POINTER(sw_scoring), U32,
                                     P, P]
        L.sw_batch_score_noalloc.argtypes = [P, ctypes.POINTER(sw_batch),
                                             ctypes.POINTER(sw_scoring), U32, P, P]
        L.sw_best_per_read.argtypes = [P, ctypes.POINTER(sw_batch), P, I32, P, P, P, P]
        L.sw_batch_traceback.argtypes = [P, ctypes.POINTER(sw_batch), ctypes.POINTER(sw_scoring),
                                         P, U32, P, P, U32, P, P]
        L.sw_select_windows.argtypes = [P, ctypes.POINTER(sw_batch), P, U32, P, P]
        L.sw_sole_windows.argtypes = [P, ctypes.POINTER(sw_batch), P, P, P, P, P]
        L.sw_merge_best.argtypes = [P, U32, P, P, P, U32, P, P]
        L.sw_cigar_string.argtypes = [P, U32, ctypes.c_char_p, U32]
        L.sw_timing_enable.argtypes = [P, ctypes.c_int]
        L.sw_ctx_set_option.argtypes = [P, ctypes.c_int, ctypes.c_int]
        L.sw_timing_get.argtypes = [P, ctypes.POINTER(sw_timing)]
        F = ctypes.c_float
        L.sw_mlp_create.argtypes = [P, ctypes.POINTER(P)]
        L.sw_mlp_destroy.argtypes = [P, P]
        L.sw_mlp_set_params.argtypes = [P, P, P]
        L.sw_mlp_get_params.argtypes = [P, P, P]
        L.sw_mlp_save.argtypes = [P, P, P, U64]
        L.sw_mlp_load.argtypes = [P, P, P, U64]
        L.sw_features.argtypes = [P, ctypes.POINTER(sw_batch), P, P]
        L.sw_mlp_forward.argtypes = [P, P, P, U32, P, P]
        L.sw_mlp_grad.argtypes = [P, P, P, P, U32, P, P, P]
        L.sw_mlp_train_step.argtypes = [P, P, P, P, U32, F, P, P]
        L.sw_mlp_labels.argtypes = [P, ctypes.POINTER(sw_batch), P, P, I32, I32, P, P]
        L.sw_filter_candidates.argtypes = [P, ctypes.POINTER(sw_batch), P,
                                           ctypes.POINTER(sw_filter_params), P, P, P, P, P, P, P, P]
        L.sw_autotune.argtypes = [P, ctypes.POINTER(sw_batch), ctypes.POINTER(sw_scoring), U32,
                                  ctypes.c_int, P, P]
        L.sw_autotune_cached.argtypes = [P, ctypes.POINTER(sw_batch), ctypes.POINTER(sw_scoring),
                                         U32, ctypes.c_int, ctypes.c_char_p,
                                         ctypes.POINTER(ctypes.c_int), P, P]
        L.sw_seed_cals.argtypes = [P, ctypes.POINTER(sw_batch), P, P, P, U32, I32, P, P]
        L.sw_join_cals.argtypes = [P, P, U32, U32, U64, U32, U32, P, P, P]
        L.sw_junctions_clear.argtypes = [P, P, P, U32, P]
        L.sw_detect_junctions.argtypes = [P, ctypes.POINTER(sw_batch), P, U32, P, P, U32, I32,
                                          U32, P, P, U32, P, P, P]
        L.sw_list_junctions.argtypes = [P, P, P, U32, P, U32, P, P]
        L.sw_kmer_index_bytes.argtypes = [U64, U32, ctypes.POINTER(ctypes.c_uint64)]
        L.sw_kmer_index_build.argtypes = [P, P, U64, U32, P, U64, P]
        L.sw_seed_regions.argtypes = [P, ctypes.POINTER(sw_batch), P, U64,
                                      ctypes.POINTER(sw_seed_params), P, U64, P, P]
        L.sw_cal_seeker.argtypes = [P, P, P, U32, U64, U32, U32, U32, P, P, P]
        L.sw_stage_b.argtypes = [P, ctypes.POINTER(sw_batch), P, P, U64, P, P, P]
        L.sw_graph_begin.argtypes = [P, P]
        L.sw_graph_end.argtypes = [P, P, ctypes.POINTER(P)]
        L.sw_graph_launch.argtypes = [P, P, P]
        L.sw_graph_destroy.argtypes = [P, P]
        for f in ("sw_ctx_create", "sw_ctx_destroy", "sw_pack2b", "sw_batch_score",
                  "sw_batch_score_noalloc",
                  "sw_best_per_read", "sw_batch_traceback", "sw_select_windows", "sw_cigar_string",
                  "sw_sole_windows", "sw_merge_best",
                  "sw_timing_enable", "sw_timing_get", "sw_ctx_set_option", "sw_mlp_create",
                  "sw_graph_begin", "sw_graph_end", "sw_graph_launch", "sw_graph_destroy",
                  "sw_autotune", "sw_autotune_cached",
                  "sw_mlp_destroy", "sw_mlp_set_params", "sw_mlp_get_params", "sw_features",
                  "sw_mlp_save", "sw_mlp_load",
                  "sw_mlp_forward", "sw_mlp_grad", "sw_mlp_train_step", "sw_mlp_labels",
                  "sw_filter_candidates", "sw_seed_cals", "sw_join_cals", "sw_junctions_clear",
                  "sw_detect_junctions", "sw_list_junctions", "sw_kmer_index_bytes",
                  "sw_kmer_index_build", "sw_seed_regions", "sw_cal_seeker", "sw_stage_b"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _stream_ptr(stream=None):
    """A torch.cuda.Stream (default: torch's current stream) as a hipStream_t."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(ctx, st):
    if st != SW_OK:
        raise SwError(st, lib().sw_last_error(ctx).decode())


def sw_ctx_create(device: int = 0):
    h = ctypes.c_void_p()
    st = lib().sw_ctx_create(device, ctypes.byref(h))
    if st != SW_OK:
        raise SwError(st, lib().sw_last_error(None).decode())
    return h


def sw_ctx_destroy(ctx):
    lib().sw_ctx_destroy(ctx)


def sw_pack2b(ctx, d_ascii, n, d_out, d_bad=None, stream=None):
    _check(ctx, lib().sw_pack2b(ctx, _ptr(d_ascii), int(n), _ptr(d_out), _ptr(d_bad),
                                _stream_ptr(stream)))


def sw_batch_score(ctx, batch, scoring, flags, d_hits, stream=None):
    _check(ctx, lib().sw_batch_score(ctx, ctypes.byref(batch.c), ctypes.byref(_sc(scoring)),
                                     int(flags), _ptr(d_hits), _stream_ptr(stream)))


def sw_batch_score_noalloc(ctx, batch, scoring, flags, d_hits, stream=None):
    """sw_batch_score on the library's static scratch (no device allocation)."""
    _check(ctx, lib().sw_batch_score_noalloc(ctx, ctypes.byref(batch.c), ctypes.byref(_sc(scoring)),
                                             int(flags), _ptr(d_hits), _stream_ptr(stream)))


def sw_best_per_read(ctx, batch, d_hits, t_map, d_best_pair, d_best_score, d_mapped=None,
                     stream=None):
    _check(ctx, lib().sw_best_per_read(ctx, ctypes.byref(batch.c), _ptr(d_hits), int(t_map),
                                       _ptr(d_best_pair), _ptr(d_best_score), _ptr(d_mapped),
                                       _stream_ptr(stream)))


def sw_select_windows(ctx, batch, d_pair_ids, n, d_win_out, stream=None):
    _check(ctx, lib().sw_select_windows(ctx, ctypes.byref(batch.c), _ptr(d_pair_ids), int(n),
                                        _ptr(d_win_out), _stream_ptr(stream)))


def sw_sole_windows(ctx, batch, d_sole, d_win_out, d_ids_out, d_n_out, stream=None):
    _check(ctx, lib().sw_sole_windows(ctx, ctypes.byref(batch.c), _ptr(d_sole), _ptr(d_win_out),
                                      _ptr(d_ids_out), _ptr(d_n_out), _stream_ptr(stream)))


def sw_merge_best(ctx, n_reads, d_sole, d_sub_best, d_ids, n_ids, d_best_pair, stream=None):
    _check(ctx, lib().sw_merge_best(ctx, int(n_reads), _ptr(d_sole), _ptr(d_sub_best), _ptr(d_ids),
                                    int(n_ids), _ptr(d_best_pair), _stream_ptr(stream)))


def sw_batch_traceback(ctx, batch, scoring, d_pair_ids, n_sel, d_aln, d_ops, ops_stride,
                       stream=None, hits=None):
    """`hits`: the batch's sw_batch_score results with SW_WANT_ENDS (optional; the
    DP then covers only the columns each alignment can reach)."""
    _check(ctx, lib().sw_batch_traceback(ctx, ctypes.byref(batch.c), ctypes.byref(_sc(scoring)),
                                         _ptr(d_pair_ids), int(n_sel), _ptr(d_aln), _ptr(d_ops),
                                         int(ops_stride), _ptr(hits), _stream_ptr(stream)))


def sw_ctx_set_option(ctx, option, value):
    _check(ctx, lib().sw_ctx_set_option(ctx, int(option), int(value)))


def sw_timing_enable(ctx, on=True):
    _check(ctx, lib().sw_timing_enable(ctx, 1 if on else 0))


def sw_timing_get(ctx) -> sw_timing:
    t = sw_timing()
    _check(ctx, lib().sw_timing_get(ctx, ctypes.byref(t)))
    return t


def sw_mlp_create(ctx):
    h = ctypes.c_void_p()
    _check(ctx, lib().sw_mlp_create(ctx, ctypes.byref(h)))
    return h


def sw_mlp_destroy(ctx, mlp):
    _check(ctx, lib().sw_mlp_destroy(ctx, mlp))


def sw_mlp_set_params(ctx, mlp, params: np.ndarray):
    a = np.ascontiguousarray(params, dtype=np.float32)
    assert a.size == SW_MLP_PARAMS
    _check(ctx, lib().sw_mlp_set_params(ctx, mlp, a.ctypes.data_as(ctypes.c_void_p)))


def sw_mlp_get_params(ctx, mlp) -> np.ndarray:
    a = np.zeros(SW_MLP_PARAMS, dtype=np.float32)
    _check(ctx, lib().sw_mlp_get_params(ctx, mlp, a.ctypes.data_as(ctypes.c_void_p)))
    return a


SW_MLP_STATE_BYTES = 24 + 12 * SW_MLP_PARAMS


def sw_mlp_save(ctx, mlp) -> bytes:
    """Checkpoint of the network and its Adam state (SW_MLP_STATE_BYTES bytes)."""
    buf = ctypes.create_string_buffer(SW_MLP_STATE_BYTES)
    _check(ctx, lib().sw_mlp_save(ctx, mlp, ctypes.cast(buf, ctypes.c_void_p), len(buf)))
    return buf.raw


def sw_mlp_load(ctx, mlp, state: bytes):
    """Restore a checkpoint written by sw_mlp_save."""
    buf = ctypes.create_string_buffer(bytes(state), len(state))
    _check(ctx, lib().sw_mlp_load(ctx, mlp, ctypes.cast(buf, ctypes.c_void_p), len(state)))


def sw_features(ctx, batch, d_feat, stream=None):
    _check(ctx, lib().sw_features(ctx, ctypes.byref(batch.c), _ptr(d_feat), _stream_ptr(stream)))


def sw_mlp_forward(ctx, mlp, d_x, n, d_logits, stream=None):
    _check(ctx, lib().sw_mlp_forward(ctx, mlp, _ptr(d_x), int(n), _ptr(d_logits),
                                     _stream_ptr(stream)))


def sw_mlp_grad(ctx, mlp, d_x, d_y, n, d_grad, d_loss, stream=None):
    _check(ctx, lib().sw_mlp_grad(ctx, mlp, _ptr(d_x), _ptr(d_y), int(n), _ptr(d_grad),
                                  _ptr(d_loss), _stream_ptr(stream)))


def sw_mlp_train_step(ctx, mlp, d_x, d_y, n, lr, d_loss=None, stream=None):
    _check(ctx, lib().sw_mlp_train_step(ctx, mlp, _ptr(d_x), _ptr(d_y), int(n), float(lr),
                                        _ptr(d_loss), _stream_ptr(stream)))


def sw_mlp_labels(ctx, batch, d_hits, d_best_score, margin, d_y, stream=None,
                  min_best=-(1 << 31)):
    _check(ctx, lib().sw_mlp_labels(ctx, ctypes.byref(batch.c), _ptr(d_hits), _ptr(d_best_score),
                                    int(margin), int(min_best), _ptr(d_y), _stream_ptr(stream)))


def sw_filter_candidates(ctx, batch, mlp, logit_lo, logit_hi, d_feat, d_logits, d_keep,
                         d_win_out, d_sel_ids, d_n_sel, d_n_unsure=None, stream=None,
                         logit_drop=float("-inf")):
    fp = sw_filter_params(float(logit_lo), float(logit_hi), float(logit_drop))
    _check(ctx, lib().sw_filter_candidates(ctx, ctypes.byref(batch.c), mlp, ctypes.byref(fp),
                                           _ptr(d_feat), _ptr(d_logits), _ptr(d_keep),
                                           _ptr(d_win_out), _ptr(d_sel_ids), _ptr(d_n_sel),
                                           _ptr(d_n_unsure), _stream_ptr(stream)))


SW_NUM_CLASSES = 11


class sw_tune_entry(ctypes.Structure):
    _fields_ = [("m_max", ctypes.c_int32), ("G", ctypes.c_int32), ("RPL", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("path", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("ms", ctypes.c_float), ("ms_default", ctypes.c_float)]


def sw_autotune(ctx, batch, scoring, flags=0, repeats=3, stream=None):
    """Tune the score kernels on a sample batch (kept in ctx); returns one dict per
    query-length class."""
    out = (sw_tune_entry * SW_NUM_CLASSES)()
    _check(ctx, lib().sw_autotune(ctx, ctypes.byref(batch.c), ctypes.byref(_sc(scoring)),
                                  int(flags), int(repeats), ctypes.cast(out, ctypes.c_void_p),
                                  _stream_ptr(stream)))
    return [{f: getattr(e, f) for f, _ in sw_tune_entry._fields_} for e in out]


def sw_autotune_cached(ctx, batch, scoring, cache_path, flags=0, repeats=3, stream=None):
    """sw_autotune through the JSON-lines cache at `cache_path`; returns
    (entries, cache_hit)."""
    out = (sw_tune_entry * SW_NUM_CLASSES)()
    hit = ctypes.c_int(0)
    _check(ctx, lib().sw_autotune_cached(ctx, ctypes.byref(batch.c), ctypes.byref(_sc(scoring)),
                                         int(flags), int(repeats), os.fsencode(cache_path),
                                         ctypes.byref(hit), ctypes.cast(out, ctypes.c_void_p),
                                         _stream_ptr(stream)))
    return [{f: getattr(e, f) for f, _ in sw_tune_entry._fields_} for e in out], bool(hit.value)


def sw_seed_cals(ctx, batch, d_best_pair, d_aln, d_seed_read, n_seeds, min_score, d_cals,
                 stream=None):
    _check(ctx, lib().sw_seed_cals(ctx, ctypes.byref(batch.c), _ptr(d_best_pair), _ptr(d_aln),
                                   _ptr(d_seed_read), int(n_seeds), int(min_score), _ptr(d_cals),
                                   _stream_ptr(stream)))


def sw_join_cals(ctx, d_cals, n_cals, n_reads, ref_len, ext, max_gap, d_win_out, d_n_out,
                 stream=None):
    _check(ctx, lib().sw_join_cals(ctx, _ptr(d_cals), int(n_cals), int(n_reads), int(ref_len),
                                   int(ext), int(max_gap), _ptr(d_win_out), _ptr(d_n_out),
                                   _stream_ptr(stream)))


def sw_junctions_clear(ctx, d_keys, d_counts, capacity, stream=None):
    _check(ctx, lib().sw_junctions_clear(ctx, _ptr(d_keys), _ptr(d_counts), int(capacity),
                                         _stream_ptr(stream)))


def sw_detect_junctions(ctx, batch, d_pair_ids, n, d_aln, d_ops, ops_stride, min_score,
                        min_intron, d_keys, d_counts, capacity, d_n_junc=None, d_dropped=None,
                        stream=None):
    _check(ctx, lib().sw_detect_junctions(ctx, ctypes.byref(batch.c), _ptr(d_pair_ids), int(n),
                                          _ptr(d_aln), _ptr(d_ops), int(ops_stride),
                                          int(min_score), int(min_intron), _ptr(d_keys),
                                          _ptr(d_counts), int(capacity), _ptr(d_n_junc),
                                          _ptr(d_dropped), _stream_ptr(stream)))


def sw_list_junctions(ctx, d_keys, d_counts, capacity, d_out, out_cap, d_n, stream=None):
    _check(ctx, lib().sw_list_junctions(ctx, _ptr(d_keys), _ptr(d_counts), int(capacity),
                                        _ptr(d_out), int(out_cap), _ptr(d_n), _stream_ptr(stream)))


def sw_kmer_index_bytes(ref_len, k) -> int:
    n = ctypes.c_uint64(0)
    st = lib().sw_kmer_index_bytes(int(ref_len), int(k), ctypes.byref(n))
    if st != SW_OK:
        raise SwError(st, lib().sw_last_error(None).decode())
    return int(n.value)


def sw_kmer_index_build(ctx, d_ref2b, ref_len, k, d_index, index_bytes, stream=None):
    _check(ctx, lib().sw_kmer_index_build(ctx, _ptr(d_ref2b), int(ref_len), int(k), _ptr(d_index),
                                          int(index_bytes), _stream_ptr(stream)))


def sw_seed_regions(ctx, batch, d_index, params, d_regions, cap, d_read_end, stream=None,
                    index_bytes=None):
    """`params`: (k, step, offset, max_occ) or sw_seed_params; `index_bytes`
    defaults to the size of the d_index tensor."""
    sp = params if isinstance(params, sw_seed_params) else sw_seed_params(*[int(x) for x in params])
    if index_bytes is None:
        index_bytes = d_index.numel() * d_index.element_size()
    _check(ctx, lib().sw_seed_regions(ctx, ctypes.byref(batch.c), _ptr(d_index), int(index_bytes),
                                      ctypes.byref(sp), _ptr(d_regions), int(cap),
                                      _ptr(d_read_end), _stream_ptr(stream)))


def sw_cal_seeker(ctx, d_regions, d_read_end, n_reads, cap, k, merge_gap, min_len, d_cals,
                  stream=None, d_skip=None):
    _check(ctx, lib().sw_cal_seeker(ctx, _ptr(d_regions), _ptr(d_read_end), int(n_reads), int(cap),
                                    int(k), int(merge_gap), int(min_len), _ptr(d_skip),
                                    _ptr(d_cals), _stream_ptr(stream)))


def sw_stage_b(ctx, batch, d_regions, d_read_end, cap, d_maps, d_n_maps, stream=None):
    _check(ctx, lib().sw_stage_b(ctx, ctypes.byref(batch.c), _ptr(d_regions), _ptr(d_read_end),
                                 int(cap), _ptr(d_maps), _ptr(d_n_maps), _stream_ptr(stream)))


def sw_graph_begin(ctx, stream):
    """Start recording the library calls issued on `stream` (a torch.cuda.Stream
    created by the caller, not the null stream)."""
    _check(ctx, lib().sw_graph_begin(ctx, _stream_ptr(stream)))


def sw_graph_end(ctx, stream):
    """Stop recording; returns a replayable graph handle."""
    g = ctypes.c_void_p()
    _check(ctx, lib().sw_graph_end(ctx, _stream_ptr(stream), ctypes.byref(g)))
    return g


def sw_graph_launch(ctx, g, stream=None):
    _check(ctx, lib().sw_graph_launch(ctx, g, _stream_ptr(stream)))


def sw_graph_destroy(ctx, g):
    _check(ctx, lib().sw_graph_destroy(ctx, g))


def sw_cigar_string(ops) -> str:
    a = np.ascontiguousarray(ops, dtype=np.uint32)
    buf = ctypes.create_string_buffer(16 * len(a) + 1)
    n = lib().sw_cigar_string(a.ctypes.data_as(ctypes.c_void_p), len(a), buf, len(buf))
    if n < 0:
        raise SwError(SW_E_INVALID, "CIGAR buffer too small")
    return buf.value.decode()


def _sc(scoring) -> sw_scoring:
    if isinstance(scoring, sw_scoring):
        return scoring
    return sw_scoring(*[int(x) for x in scoring])


class DeviceBatch:
    """A batch resident in device memory: packed reference, packed reads, windows.

    Built from ASCII host arrays; the 2-bit encoding runs on the device through
    sw_pack2b.  Keeps the torch tensors alive as long as the batch exists.
    """

    def __init__(self, ctx, ref_ascii, reads_ascii, read_off, read_len, windows, stream=None,
                 ref2b=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        self.ctx = ctx
        self.bad = torch.zeros(1, dtype=torch.int32, device=dev)
        if ref2b is None:
            self.ref_ascii = torch.from_numpy(np.ascontiguousarray(ref_ascii)).to(dev)
            self.ref2b = torch.empty((len(ref_ascii) + 15) // 16, dtype=torch.int32, device=dev)
            sw_pack2b(ctx, self.ref_ascii, len(ref_ascii), self.ref2b, self.bad, stream)
            self.ref_len = len(ref_ascii)
        else:
            self.ref2b, self.ref_len = ref2b
        self.reads_ascii = torch.from_numpy(np.ascontiguousarray(reads_ascii)).to(dev)
        self.reads_len = len(reads_ascii)
        self.reads2b = torch.empty(max((self.reads_len + 15) // 16, 1), dtype=torch.int32,
                                   device=dev)
        self.read_off = torch.from_numpy(np.ascontiguousarray(read_off, dtype=np.uint64)
                                         .view(np.int64)).to(dev)
        self.read_len = torch.from_numpy(np.ascontiguousarray(read_len, dtype=np.uint16)
                                         .view(np.int16)).to(dev)
        w = np.ascontiguousarray(windows).view(np.uint8)
        self.win = torch.from_numpy(w.copy()).to(dev)
        self.n_reads = len(read_len)
        self.n_pairs = len(windows)
        self.read_len_max = int(np.max(read_len, initial=0))
        self.window_len_max = int(np.max(np.asarray(windows)["len"], initial=0)) if len(windows) else 0
        self.pack_reads(stream)
        self.c = sw_batch(_ptr(self.ref2b), self.ref_len, _ptr(self.reads2b), self.reads_len,
                          _ptr(self.read_off), _ptr(self.read_len), self.n_reads, _ptr(self.win),
                          self.n_pairs, None)

    def view(self, win, n_pairs, d_n_pairs=None):
        """The same reads and reference with another window list (e.g. a
        compacted work list whose count stays on the device)."""
        v = object.__new__(DeviceBatch)
        v.__dict__.update(self.__dict__)
        v.win_view = win
        v.n_pairs = n_pairs
        v.c = sw_batch(_ptr(self.ref2b), self.ref_len, _ptr(self.reads2b), self.reads_len,
                       _ptr(self.read_off), _ptr(self.read_len), self.n_reads, _ptr(win),
                       n_pairs, _ptr(d_n_pairs))
        return v

    def pack_reads(self, stream=None):
        """Encode step for the reads (ASCII already in device memory)."""
        sw_pack2b(self.ctx, self.reads_ascii, self.reads_len, self.reads2b, self.bad, stream)

    @classmethod
    def from_synth(cls, ctx, b, stream=None):
        return cls(ctx, b.ref, b.reads, b.read_off, b.read_len, b.windows, stream)


def hits_to_numpy(t) -> np.ndarray:
    return t.cpu().numpy().view(HIT_DTYPE).reshape(-1)


def aln_to_numpy(t) -> np.ndarray:
    return t.cpu().numpy().view(ALN_DTYPE).reshape(-1)


def junctions_to_numpy(t) -> np.ndarray:
    return t.cpu().numpy().view(JUNCTION_DTYPE).reshape(-1)
