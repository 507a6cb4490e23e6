"""A plain device-to-device copy of a known size (256 MiB, three times), for
scaling hardware byte counters (FETCH_SIZE, WRITE_SIZE) to bytes moved: the
counters of this copy are compared with 3 x 256 MiB read and written.

  python -m paper_1807_01350_amd.copy_probe
"""
import torch


def main():
    n = 64 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied", n * 4, "bytes x 3")


if __name__ == "__main__":
    main()
