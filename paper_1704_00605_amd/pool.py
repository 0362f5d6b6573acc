"""Device memory pool: one torch allocation managed by the library's buddy
allocator (``b64_pool_*`` in ``include/b64.h``). ``try_alloc`` never blocks:
it returns None when no block is free, which the serving loop uses for
admission by free HBM."""
import ctypes

from ._lib import OK, POOL_FULL, check, lib


class BuddyPool:
    """Host bookkeeping of offsets in [0, capacity) (no device memory)."""

    def __init__(self, capacity, min_block=256):
        h = ctypes.c_void_p()
        check(lib().b64_pool_create(int(capacity), int(min_block), ctypes.byref(h)), "b64_pool_create")
        self.handle = h
        self.capacity = int(capacity)
        self.min_block = int(min_block)

    def try_alloc(self, nbytes):
        off = ctypes.c_int64(-1)
        rc = lib().b64_pool_alloc(self.handle, int(nbytes), ctypes.byref(off))
        if rc == POOL_FULL:
            return None
        check(rc, "b64_pool_alloc")
        return off.value

    def free(self, offset):
        check(lib().b64_pool_free(self.handle, int(offset)), "b64_pool_free")

    def free_bytes(self):
        return check(lib().b64_pool_free_bytes(self.handle), "b64_pool_free_bytes")

    def peak_bytes(self):
        return check(lib().b64_pool_peak_bytes(self.handle), "b64_pool_peak_bytes")

    def close(self):
        if self.handle:
            lib().b64_pool_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DevicePool(BuddyPool):
    """A buddy pool over one uint8 CUDA tensor of ``capacity`` bytes."""

    def __init__(self, capacity, device="cuda:0", min_block=256):
        import torch

        super().__init__(capacity, min_block)
        self.buf = torch.empty(int(capacity), dtype=torch.uint8, device=device)

    def base_ptr(self):
        return self.buf.data_ptr()

    def view(self, offset, nbytes):
        return self.buf[offset:offset + nbytes]


__all__ = ["BuddyPool", "DevicePool", "OK", "POOL_FULL"]
