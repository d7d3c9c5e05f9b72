"""Quotient jobs with host-resident inputs and outputs, PCIe transfers
overlapped with compute.

The paper finds that for GPU NTTs the host-device transfers take longer than
the transforms and are not hidden (Section IV-A, the compute-versus-memory
breakdown; Section IV-C).  This pipeline keeps `depth` device slots per size
and drives three streams, so that the copy engines and the compute units work
at the same time:

    h2d stream      A_k -> slot, event; B_k -> slot, event; C_k -> slot, event
    compute stream  waits for A_k: quotient_coset_evals(A_k)   (overlaps B_k's copy)
                    waits for B_k: quotient_coset_evals(B_k)   (overlaps C_k's copy)
                    waits for C_k: quotient_coset_evals(C_k), quotient_pointwise,
                                   ntt_coset_inverse -> H_k, event
    d2h stream      waits for H_k: H_k -> host (zk_copy_to_host), event frees
                    the slot

Job k + 1's uploads run while job k computes and job k - 1 downloads.  The
uploads are DMA copies and the download is a copy kernel storing into the
pinned host buffer: measured on MI355X, two DMA copies in opposite
directions ran one after the other, while a DMA upload and the kernel
download run at the same time, so both directions of the link are busy.  Every
stage is a call of the C library on device buffers; the pipeline only orders
them with events.  Results equal quotient_poly byte for byte.

Host buffers must be pinned (torch's pin_memory allocates them) for the
copies to be asynchronous.
"""
from __future__ import annotations

import dataclasses


@dataclasses.dataclass
class _Slot:
    A: object
    B: object
    C: object
    work: object
    free: object  # event: the slot's previous download has finished


class HostQuotientPipeline:
    def __init__(self, field: str = "bls12_381_fr", device=None, depth: int = 2):
        import torch

        self.torch = torch
        self.field = field
        self.device = torch.device(device or "cuda:0")
        self.depth = depth
        self.h2d = torch.cuda.Stream(self.device)
        self.compute = torch.cuda.Stream(self.device)
        self.d2h = torch.cuda.Stream(self.device)
        self.plans = {}
        self.slots = {}
        self.next_slot = {}

    def plan(self, log2n: int):
        from ._lib import Plan

        if log2n not in self.plans:
            with self.torch.cuda.device(self.device):
                self.plans[log2n] = Plan(self.field, log2n)
        return self.plans[log2n]

    def _slot(self, log2n: int) -> _Slot:
        from ._lib import ntt_workspace_bytes

        torch = self.torch
        if log2n not in self.slots:
            n = 1 << log2n
            p = self.plan(log2n)
            wb = ntt_workspace_bytes(p.handle)
            slots = []
            for _ in range(self.depth):
                bufs = torch.empty(3 * n, 8, dtype=torch.int32, device=self.device)
                work = torch.empty(max(wb, 32) // 32, 8, dtype=torch.int32, device=self.device) if wb else None
                ev = torch.cuda.Event()
                ev.record(self.d2h)
                slots.append(_Slot(bufs[:n], bufs[n:2 * n], bufs[2 * n:], work, ev))
            self.slots[log2n] = slots
            self.next_slot[log2n] = 0
        k = self.next_slot[log2n]
        self.next_slot[log2n] = (k + 1) % self.depth
        return self.slots[log2n][k]

    def submit(self, A, B, C, H):
        """Queue one job: A, B, C pinned host tensors [n, 8] int32 (Montgomery
        limbs), H a pinned host tensor that receives the result.  Returns the
        event that marks H complete."""
        from ._lib import ntt_coset_inverse, quotient_coset_evals, quotient_pointwise, zk_copy_to_host

        torch = self.torch
        n = A.shape[0]
        log2n = n.bit_length() - 1
        if n != 1 << log2n or B.shape != A.shape or C.shape != A.shape or H.shape != A.shape:
            raise ValueError("A, B, C, H must be [n, 8] with n a power of two")
        p = self.plan(log2n)
        s = self._slot(log2n)
        arrived = []
        self.h2d.wait_event(s.free)
        with torch.cuda.stream(self.h2d):
            for dst, src in ((s.A, A), (s.B, B), (s.C, C)):
                dst.copy_(src, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self.h2d)
                arrived.append(ev)
        cs = self.compute
        for ev, buf in zip(arrived, (s.A, s.B, s.C)):
            cs.wait_event(ev)
            quotient_coset_evals(p.handle, buf, buf, s.work, cs)
        quotient_pointwise(p.handle, s.A, s.B, s.C, s.C, cs)
        ntt_coset_inverse(p.handle, s.C, s.C, s.work, cs)
        ready = torch.cuda.Event()
        ready.record(cs)
        self.d2h.wait_event(ready)
        zk_copy_to_host(H, s.C, n * 32, self.d2h)
        done = torch.cuda.Event()
        done.record(self.d2h)
        s.free = done
        # the slot's device buffers are reused only after `done`; keep the
        # host tensors alive until then as well
        return done

    def run_serial(self, A, B, C, H) -> None:
        """The same job with nothing overlapped: upload, compute, download,
        each waited for (the reference the pipeline is measured against)."""
        from ._lib import ntt_coset_inverse, quotient_coset_evals, quotient_pointwise

        torch = self.torch
        n = A.shape[0]
        log2n = n.bit_length() - 1
        p = self.plan(log2n)
        s = self._slot(log2n)
        s.free.synchronize()
        for dst, src in ((s.A, A), (s.B, B), (s.C, C)):
            dst.copy_(src)
        torch.cuda.synchronize(self.device)
        cs = torch.cuda.current_stream(self.device)
        for buf in (s.A, s.B, s.C):
            quotient_coset_evals(p.handle, buf, buf, s.work, cs)
        quotient_pointwise(p.handle, s.A, s.B, s.C, s.C, cs)
        ntt_coset_inverse(p.handle, s.C, s.C, s.work, cs)
        torch.cuda.synchronize(self.device)
        H.copy_(s.C)
        torch.cuda.synchronize(self.device)
