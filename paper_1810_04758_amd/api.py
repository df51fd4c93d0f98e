"""Python surface of the library (same names as the C ABI in include/knnjoin.h).

PyTorch is used only for device memory and streams: device tensors are passed
to the HIP library as raw pointers, and the library runs every step.
"""

import ctypes

import numpy as np

from . import _lib
from ._lib import (BuildOpts, EpsConsumer, EpsJoinStats, HybridOpts, HybridStats, IndexInfo,
                   JoinOpts, JoinStats, ServerOpts, ServerStats, check, load)


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _join_opts(w_factor=0.0, cell_width=0.0, lanes_per_query=0, schedule=0, batch_queries=0,
               eps_step=0.0, linear_levels=0, growth=0.0, use_graph=0, tail_pairs=0.0,
               heavy_min=0, queue_grain=0, item_order=0, lanes_shift=0, share_lists=0,
               speculate=0, predict_fail=0, zorder=0,
               stats=None):
    o = JoinOpts()
    load().knn_join_opts_default(ctypes.byref(o))
    o.w_factor = w_factor
    o.cell_width = cell_width
    o.lanes_per_query = lanes_per_query
    o.schedule = schedule
    o.batch_queries = batch_queries
    o.eps_step = eps_step
    o.linear_levels = linear_levels
    o.growth = growth
    o.use_graph = use_graph
    o.tail_pairs = tail_pairs
    o.heavy_min = heavy_min
    o.queue_grain = queue_grain
    o.item_order = item_order
    o.lanes_shift = lanes_shift
    o.share_lists = share_lists
    o.speculate = speculate
    o.predict_fail = predict_fail
    o.zorder = zorder
    o.stats = ctypes.pointer(stats) if stats is not None else None
    return o


def _build_opts(seed=1, n_sample=0, n_bins=0, mean_frac=0.0, min_mean_sample=0, device=-1):
    o = BuildOpts()
    load().knn_build_opts_default(ctypes.byref(o))
    o.seed = seed
    o.n_sample = n_sample
    o.n_bins = n_bins
    o.mean_frac = mean_frac
    o.min_mean_sample = min_mean_sample
    o.device = device
    return o


class Index:
    """A dataset resident in device memory (knn_index)."""

    def __init__(self, handle, N, dims):
        self._h = handle
        self.N = N
        self.dims = dims

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("index is closed")
        return self._h

    def close(self):
        if self._h is not None:
            load().knn_destroy_index(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        inf = IndexInfo()
        check(load().knn_index_info_get(self.handle, ctypes.byref(inf)))
        n = inf.dims
        return dict(n_points=inf.n_points, dims=n, device=inf.device, lo=list(inf.lo[:n]),
                    hi=list(inf.hi[:n]), eps_mean=inf.eps_mean, n_bins=inf.n_bins,
                    n_sample=inf.n_sample, device_bytes=inf.device_bytes)

    def eps_min(self, K):
        v = ctypes.c_double()
        check(load().knn_eps_min(self.handle, K, ctypes.byref(v)))
        return v.value

    def sampling(self):
        """knn_index_sampling_get: the index's Sec. 4.4 samples and histogram
        (histogram sample ids, eps_mean sample ids, per-bin counts, bin width)."""
        inf = self.info()
        hs = np.empty(inf["n_sample"], dtype=np.int64)
        ms = np.empty(20000, dtype=np.int64)
        counts = np.empty(inf["n_bins"], dtype=np.uint64)
        nm = ctypes.c_int64()
        bw = ctypes.c_double()
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        check(load().knn_index_sampling_get(self.handle, p(hs), p(ms), ctypes.byref(nm),
                                            p(counts), ctypes.byref(bw)))
        return dict(hist_sample=hs, mean_sample=ms[:nm.value].copy(), counts=counts,
                    bin_width=bw.value)

    def autotune(self, K, stream=None):
        """knn_autotune: measure and cache the best (w_factor, growth) for K."""
        r = _lib.AutotuneResult()
        check(load().knn_autotune(self.handle, K, _stream_ptr(stream), ctypes.byref(r)))
        return {f: getattr(r, f) for f, _ in _lib.AutotuneResult._fields_}

    def join_footprint(self, K):
        """knn_join_footprint: device bytes a host-output join of K allocates."""
        v = ctypes.c_uint64()
        check(load().knn_join_footprint(self.handle, K, ctypes.byref(v)))
        return v.value

    def self_join(self, K, ids=None, dists=None, stream=None, with_stats=False, **opts):
        """knn_self_join_device: returns (ids int32 [N,K], dists float64 [N,K]) on
        the GPU (and the per-level statistics if with_stats)."""
        torch = _torch()
        dev = torch.device("cuda", torch.cuda.current_device())
        if ids is None:
            ids = torch.empty((self.N, K), dtype=torch.int32, device=dev)
        if dists is None:
            dists = torch.empty((self.N, K), dtype=torch.float64, device=dev)
        if ids.shape != (self.N, K) or dists.shape != (self.N, K):
            raise ValueError("output shape must be (N, K)")
        if ids.dtype != torch.int32 or dists.dtype != torch.float64:
            raise ValueError("outputs must be int32 / float64")
        if not (ids.is_cuda and dists.is_cuda and ids.is_contiguous() and dists.is_contiguous()):
            raise ValueError("outputs must be contiguous device tensors")
        st = JoinStats() if with_stats else None
        o = _join_opts(stats=st, **opts)
        check(load().knn_self_join_device(self.handle, K, ctypes.c_void_p(ids.data_ptr()),
                                          ctypes.c_void_p(dists.data_ptr()), ctypes.byref(o),
                                          _stream_ptr(stream)))
        if with_stats:
            return ids, dists, st.as_dict()
        return ids, dists

    def join(self, Q, K, ids=None, dists=None, stream=None, with_stats=False, **opts):
        """knn_join_device / knn_join: the K nearest points of the index for
        every row of Q (R join S of Sec. 2.1, nothing excluded).  Q: a CUDA
        tensor (results on the device) or a numpy array (results on the
        host), n_queries x dims float64."""
        st = JoinStats() if with_stats else None
        o = _join_opts(stats=st, **opts)
        torch = _torch()
        if Q.shape[-1] != self.dims:
            raise ValueError("Q must have the index's number of dimensions")
        if isinstance(Q, torch.Tensor) and Q.is_cuda:
            if Q.dtype != torch.float64 or Q.dim() != 2 or not Q.is_contiguous():
                raise ValueError("Q must be a contiguous float64 n_queries x dims tensor")
            NQ = Q.shape[0]
            if ids is None:
                ids = torch.empty((NQ, K), dtype=torch.int32, device=Q.device)
            if dists is None:
                dists = torch.empty((NQ, K), dtype=torch.float64, device=Q.device)
            if ids.shape != (NQ, K) or dists.shape != (NQ, K):
                raise ValueError("output shape must be (n_queries, K)")
            check(load().knn_join_device(self.handle, ctypes.c_void_p(Q.data_ptr()), NQ, K,
                                         ctypes.c_void_p(ids.data_ptr()),
                                         ctypes.c_void_p(dists.data_ptr()), ctypes.byref(o),
                                         _stream_ptr(stream)))
        else:
            Qh = np.ascontiguousarray(Q.numpy() if isinstance(Q, torch.Tensor) else Q,
                                      dtype=np.float64)
            if Qh.ndim != 2:
                raise ValueError("Q must be n_queries x dims")
            NQ = Qh.shape[0]
            ids = np.empty((NQ, K), dtype=np.int32)
            dists = np.empty((NQ, K), dtype=np.float64)
            check(load().knn_join(self.handle, Qh.ctypes.data_as(ctypes.c_void_p), NQ, K,
                                  ids.ctypes.data_as(ctypes.c_void_p),
                                  dists.ctypes.data_as(ctypes.c_void_p), ctypes.byref(o)))
        if with_stats:
            return ids, dists, st.as_dict()
        return ids, dists

    def self_join_noalloc(self, K, ids, dists, stream=None, **opts):
        """knn_self_join_device_noalloc: the same join with every temporary in
        the library's fixed scratch area (no device allocation); ids / dists
        are caller-provided contiguous device tensors (N x K int32 / float64)."""
        torch = _torch()
        if ids.shape != (self.N, K) or dists.shape != (self.N, K):
            raise ValueError("output shape must be (N, K)")
        if ids.dtype != torch.int32 or dists.dtype != torch.float64:
            raise ValueError("outputs must be int32 / float64")
        if not (ids.is_cuda and dists.is_cuda and ids.is_contiguous() and dists.is_contiguous()):
            raise ValueError("outputs must be contiguous device tensors")
        o = _join_opts(**opts)
        check(load().knn_self_join_device_noalloc(self.handle, K, ctypes.c_void_p(ids.data_ptr()),
                                                  ctypes.c_void_p(dists.data_ptr()),
                                                  ctypes.byref(o), _stream_ptr(stream)))
        return ids, dists

    def self_join_host(self, K, with_stats=False, **opts):
        """knn_self_join: results in host (numpy) arrays."""
        ids = np.empty((self.N, K), dtype=np.int32)
        dists = np.empty((self.N, K), dtype=np.float64)
        st = JoinStats() if with_stats else None
        o = _join_opts(stats=st, **opts)
        check(load().knn_self_join(self.handle, K, ids.ctypes.data_as(ctypes.c_void_p),
                                   dists.ctypes.data_as(ctypes.c_void_p), ctypes.byref(o)))
        if with_stats:
            return ids, dists, st.as_dict()
        return ids, dists

    def self_join_hybrid(self, K, n_large=0.0, n_small=0.0, n_cwin=0.0, n_cpu=0.0,
                         eps_factor=0.0, cpu_threads=0, zorder=0):
        """knn_self_join_hybrid: the KNN self-join split between the GPU (dense
        end of the work queue) and host threads (sparse end).  Returns
        (ids int32 [N,K], dists float64 [N,K], stats dict) in host memory."""
        ids = np.empty((self.N, K), dtype=np.int32)
        dists = np.empty((self.N, K), dtype=np.float64)
        o = HybridOpts(n_large=n_large, n_small=n_small, n_cwin=n_cwin, n_cpu=n_cpu,
                       eps_factor=eps_factor, cpu_threads=cpu_threads, zorder=zorder)
        st = HybridStats()
        check(load().knn_self_join_hybrid(self.handle, K, ids.ctypes.data_as(ctypes.c_void_p),
                                          dists.ctypes.data_as(ctypes.c_void_p), ctypes.byref(o),
                                          ctypes.byref(st)))
        return ids, dists, {f: getattr(st, f) for f, _ in HybridStats._fields_}

    # ---- distance similarity self-join (every pair within eps) ----------------

    def eps_join_size(self, eps, sample_stride=1, counts=False, stream=None):
        """knn_eps_join_size: the exact number of pairs within eps
        (sample_stride 1; with counts=True also the pairs of each point id, an
        int32 device tensor of N entries), or the sampled estimate
        (sample_stride > 1).  Returns n_pairs or (n_pairs, counts)."""
        torch = _torch()
        n = ctypes.c_uint64()
        c = None
        if counts:
            c = torch.empty(self.N, dtype=torch.int32,
                            device=torch.device("cuda", torch.cuda.current_device()))
        check(load().knn_eps_join_size(self.handle, float(eps), int(sample_stride),
                                       ctypes.byref(n),
                                       ctypes.c_void_p(c.data_ptr() if c is not None else 0),
                                       _stream_ptr(stream)))
        return (n.value, c) if counts else n.value

    def eps_join_batch(self, eps, cursor, qids, nids, dists, stream=None):
        """knn_eps_join_device: the next batch from `cursor` into the device
        tensors qids / nids (int32) and dists (float64), whose common length is
        the capacity.  Returns (n_pairs, next_cursor)."""
        torch = _torch()
        cap = qids.numel()
        if nids.numel() != cap or dists.numel() != cap:
            raise ValueError("qids, nids and dists must have the same length")
        if qids.dtype != torch.int32 or nids.dtype != torch.int32 or dists.dtype != torch.float64:
            raise ValueError("qids / nids must be int32 and dists float64")
        for t in (qids, nids, dists):
            if not (t.is_cuda and t.is_contiguous()):
                raise ValueError("outputs must be contiguous device tensors")
        n = ctypes.c_uint64()
        nxt = ctypes.c_int64()
        check(load().knn_eps_join_device(self.handle, float(eps), int(cursor), cap,
                                         ctypes.c_void_p(qids.data_ptr()),
                                         ctypes.c_void_p(nids.data_ptr()),
                                         ctypes.c_void_p(dists.data_ptr()), ctypes.byref(n),
                                         ctypes.byref(nxt), _stream_ptr(stream)))
        return n.value, nxt.value

    def eps_join_device(self, eps, capacity=0, stream=None):
        """Every pair within eps on the device, batch by batch (capacity pairs
        per batch; 0: the exact total, one batch).  Returns (qids, nids, dists)
        device tensors holding all pairs, in batch order."""
        torch = _torch()
        dev = torch.device("cuda", torch.cuda.current_device())
        total = self.eps_join_size(eps, stream=stream)
        cap = capacity if capacity > 0 else max(total, 1)
        q = torch.empty(total, dtype=torch.int32, device=dev)
        j = torch.empty(total, dtype=torch.int32, device=dev)
        d = torch.empty(total, dtype=torch.float64, device=dev)
        bq = torch.empty(cap, dtype=torch.int32, device=dev)
        bj = torch.empty(cap, dtype=torch.int32, device=dev)
        bd = torch.empty(cap, dtype=torch.float64, device=dev)
        cursor, at = 0, 0
        while cursor < self.N:
            n, cursor = self.eps_join_batch(eps, cursor, bq, bj, bd, stream=stream)
            q[at:at + n].copy_(bq[:n])
            j[at:at + n].copy_(bj[:n])
            d[at:at + n].copy_(bd[:n])
            at += n
        if at != total:
            raise RuntimeError(f"batches held {at} pairs, the count pass {total}")
        return q, j, d

    def eps_join(self, eps, consume=None, batch_pairs=0, n_streams=0):
        """knn_eps_join: every pair within eps streamed to host memory in
        batches.  consume(qids, nids, dists) gets numpy views valid during the
        call (return True to stop); without it the pairs are gathered and
        returned as (qids, nids, dists, stats)."""
        parts = []

        def _cb(q, j, d, n, _user):
            n = int(n)
            qa = np.ctypeslib.as_array(q, shape=(n,)) if n else np.empty(0, np.int32)
            ja = np.ctypeslib.as_array(j, shape=(n,)) if n else np.empty(0, np.int32)
            da = np.ctypeslib.as_array(d, shape=(n,)) if n else np.empty(0, np.float64)
            if consume is None:
                parts.append((qa.copy(), ja.copy(), da.copy()))
                return 0
            return 1 if consume(qa, ja, da) else 0

        cb = EpsConsumer(_cb)
        st = EpsJoinStats()
        check(load().knn_eps_join(self.handle, float(eps), int(batch_pairs), int(n_streams), cb,
                                  None, ctypes.byref(st)))
        stats = {f: getattr(st, f) for f, _ in EpsJoinStats._fields_}
        if consume is not None:
            return stats
        if parts:
            q, j, d = (np.concatenate([p[i] for p in parts]) for i in range(3))
        else:
            q, j, d = (np.empty(0, np.int32), np.empty(0, np.int32), np.empty(0, np.float64))
        return q, j, d, stats

    def eps_join_release(self):
        """knn_eps_join_release: frees the level and counts kept for the last eps."""
        check(load().knn_eps_join_release(self.handle))

    def grid_export(self, cell_width):
        """knn_grid_export: the grid level of the given cell side, on the host."""
        N, n = self.N, self.dims
        R = 3 ** (n - 1)
        sk = np.empty(N, dtype=np.uint64)
        perm = np.empty(N, dtype=np.int32)
        ck = np.empty(N, dtype=np.uint64)
        cs = np.empty(N + 1, dtype=np.uint32)
        rg = np.empty(N * R * 2, dtype=np.uint32)
        gd = np.empty(n, dtype=np.int64)
        M = ctypes.c_int64()
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        check(load().knn_grid_export(self.handle, cell_width, p(sk), p(perm), p(ck), p(cs),
                                     p(rg), p(gd), ctypes.byref(M)))
        M = M.value
        return dict(sorted_keys=sk, perm=perm, cell_keys=ck[:M].copy(),
                    cell_start=cs[:M + 1].astype(np.int64), g=gd,
                    ranges=rg[:M * R * 2].reshape(M, R, 2).astype(np.int64))


def build_index(D, seed=1, stream=None, **kw):
    """knn_build_index / knn_build_index_device.  D: N x dims float64, either a
    numpy array (host) or a CUDA tensor (device)."""
    h = ctypes.c_void_p()
    o = _build_opts(seed=seed, **kw)
    try:
        torch = _torch()
        is_dev = isinstance(D, torch.Tensor) and D.is_cuda
    except ImportError:
        torch = None
        is_dev = False
    if is_dev:
        if D.dtype != torch.float64 or D.dim() != 2 or not D.is_contiguous():
            raise ValueError("D must be a contiguous float64 N x dims tensor")
        N, n = D.shape
        check(load().knn_build_index_device(ctypes.c_void_p(D.data_ptr()), N, n,
                                            ctypes.byref(o), _stream_ptr(stream), ctypes.byref(h)))
    else:
        if torch is not None and isinstance(D, torch.Tensor):
            D = D.numpy()
        D = np.ascontiguousarray(D, dtype=np.float64)
        if D.ndim != 2:
            raise ValueError("D must be N x dims")
        N, n = D.shape
        check(load().knn_build_index(D.ctypes.data_as(ctypes.c_void_p), N, n, ctypes.byref(o),
                                     ctypes.byref(h)))
    return Index(h, N, n)


def sample_mean_dist(D, sample, stream=None):
    """knn_sample_mean_dist on device tensors (D N x n float64, sample int64)."""
    torch = _torch()
    D = D.contiguous()
    sample = sample.to(torch.int64).contiguous()
    out = ctypes.c_double()
    check(load().knn_sample_mean_dist(ctypes.c_void_p(D.data_ptr()), D.shape[0], D.shape[1],
                                      ctypes.c_void_p(sample.data_ptr()), sample.numel(),
                                      ctypes.byref(out), _stream_ptr(stream)))
    return out.value


def dist_histogram(D, sample, inv_bin_width, n_bins, stream=None):
    """knn_dist_histogram on device tensors; returns a uint64 counts tensor."""
    torch = _torch()
    D = D.contiguous()
    sample = sample.to(torch.int64).contiguous()
    counts = torch.empty(n_bins, dtype=torch.int64, device=D.device)  # uint64 bits
    check(load().knn_dist_histogram(ctypes.c_void_p(D.data_ptr()), D.shape[0], D.shape[1],
                                    ctypes.c_void_p(sample.data_ptr()), sample.numel(),
                                    inv_bin_width, n_bins, ctypes.c_void_p(counts.data_ptr()),
                                    _stream_ptr(stream)))
    return counts


class Server:
    """knn_server_*: continuous-batching request loop over resident indexes."""

    def __init__(self, mem_budget_bytes=0, max_inflight=0, max_queue=0, device=-1):
        o = ServerOpts(mem_budget_bytes, max_inflight, max_queue, device)
        h = ctypes.c_void_p()
        check(load().knn_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def add_dataset(self, index):
        ds = ctypes.c_int32()
        check(load().knn_server_add_dataset(self._h, index.handle, ctypes.byref(ds)))
        return ds.value

    def submit(self, dataset, K, N, discard=False):
        """knn_server_submit; discard=True makes a latency-only request."""
        t = ctypes.c_int64()
        if discard:
            check(load().knn_server_submit(self._h, dataset, K, None, None, ctypes.byref(t)))
            self._keep[t.value] = (None, None)
            return t.value
        ids = np.empty((N, K), dtype=np.int32)
        dists = np.empty((N, K), dtype=np.float64)
        check(load().knn_server_submit(self._h, dataset, K, ids.ctypes.data_as(ctypes.c_void_p),
                                       dists.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t)))
        self._keep[t.value] = (ids, dists)
        return t.value

    def wait(self, ticket, timeout_us=-1):
        check(load().knn_server_wait(self._h, ticket, timeout_us))
        return self._keep.pop(ticket)

    def stats(self):
        s = ServerStats()
        check(load().knn_server_stats_get(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._h is not None:
            load().knn_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_save(path=None):
    """knn_autotune_save: write the autotune cache (path None: $KNN_AUTOTUNE_CACHE)."""
    check(load().knn_autotune_save(path.encode() if path else None))


def autotune_load(path=None):
    """knn_autotune_load: read an autotune cache file."""
    check(load().knn_autotune_load(path.encode() if path else None))
