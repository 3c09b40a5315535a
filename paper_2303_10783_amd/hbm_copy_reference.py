"""Reference traffic for hardware counters: a plain device-to-device copy of
a known size (256 MiB read + 256 MiB written per launch), launched 5 times.
Run under rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) to obtain the counter
value of a kernel whose HBM bytes are known; the ratio calibrates the
counters read for the solver kernels."""
import torch

N = 32 * 1024 * 1024            # FP64 values: 256 MiB
a = torch.rand(N, dtype=torch.float64, device="cuda")
b = torch.empty_like(a)
torch.cuda.synchronize()
for _ in range(5):
    b.copy_(a)
torch.cuda.synchronize()
print("copied", N * 8, "bytes per launch")
