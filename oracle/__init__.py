"""CPU oracle for the QDS + Klein-Gordon field advance.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``; never by the product path.
"""
