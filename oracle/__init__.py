"""FP64 CPU oracle (test infrastructure only; see ``dvbm_oracle``)."""
