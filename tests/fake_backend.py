"""A serving backend that runs the serial oracle on the CPU: the test double behind which the
scheduler's admission, memory accounting, batching and failure handling are tested without a
GPU.  Test infrastructure only (it loads the oracle)."""
from oracle import oracle as O
from paper_1508_03235_amd.serve import Backend


class OracleBackend(Backend):
    """The serial oracle behind the same interface (test double for the scheduler)."""

    def __init__(self):
        self.O = O

    def state_bytes(self, params) -> int:
        N = params.tiles
        return N * (128 + 96 + 16 + 4 * (params.l1_sets * params.l1_ways + params.l2_sets * params.l2_ways))

    def create(self, params):
        return self.O.OracleSim(params)

    def step(self, chips, cycles):
        for c, n in zip(chips, cycles):
            self.step_one(c, n)

    def step_one(self, chip, cycles):
        if cycles:
            chip.step(int(cycles))

    def cycle(self, chip):
        return chip.cycle

    def check(self, chip):
        pass

    def stats(self, chip):
        return chip.stats()

    def release(self, chip):
        chip.close()
